// Table build (FP64) for the Monte Carlo transport: spectral bins, source
// spectrum, extinction, species choice, emission E_s(T_k) and the
// difference-emissivity rows used to pick the re-emission frequency
// (paper Sec. 2: the new frequency follows from the cell temperature before
// the absorption).  Also leaf levels, FP32 copies and an input check.
#include <float.h>

#include "mcrt_internal.h"

namespace mcrt {

namespace {

__global__ void k_lambda(int nl, int S, int K, const double* __restrict__ lam_um,
                         const double* __restrict__ kabs, const double* __restrict__ ksca,
                         const double* __restrict__ g, const int32_t* __restrict__ kind,
                         double teff, double T_lo, double T_hi, double* nu, double* dnu,
                         double* src_cdf, double* kext, double* albedo, double* gpar,
                         double* sp_cdf, double* Tk, float* kext32, float* g32,
                         int32_t* pah_slot) {
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    // bin edges at geometric midpoints; outer edges half a log step out
    const double lam = lam_um[j] * 1e-4;
    const double lo = (j > 0 ? sqrt(lam_um[j - 1] * lam_um[j])
                             : lam_um[0] * lam_um[0] / sqrt(lam_um[0] * lam_um[1])) * 1e-4;
    const double hi = (j < nl - 1 ? sqrt(lam_um[j] * lam_um[j + 1])
                                  : lam_um[nl - 1] * lam_um[nl - 1] / sqrt(lam_um[nl - 2] * lam_um[nl - 1])) * 1e-4;
    nu[j] = kC / lam;
    dnu[j] = kC / lo - kC / hi;
    double ka = 0.0, ks = 0.0;
    for (int s = 0; s < S; ++s) { ka += kabs[s * nl + j]; ks += ksca[s * nl + j]; }
    kext[j] = ka + ks;
    albedo[j] = (ka + ks) > 0.0 ? ks / (ka + ks) : 0.0;
    gpar[j] = g[j];
    kext32[j] = (float)(ka + ks);
    g32[j] = (float)g[j];
    double cum = 0.0;
    for (int s = 0; s < S; ++s) {
      cum += kabs[s * nl + j];
      sp_cdf[(int64_t)j * S + s] = ka > 0.0 ? cum / ka : 1.0;
    }
    sp_cdf[(int64_t)j * S + S - 1] = 1.0;
  }
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    Tk[k] = T_lo * pow(T_hi / T_lo, (double)k / (double)(K - 1));
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int j = 0; j < nl; ++j) { tot += planck_nu(nu[j], teff) * dnu[j]; src_cdf[j] = tot; }
    for (int j = 0; j < nl; ++j) src_cdf[j] /= tot;
    src_cdf[nl - 1] = 1.0;
    int np = 0;
    for (int s = 0; s < S; ++s) pah_slot[s] = kind[s] == 1 ? np++ : -1;
  }
}

// B_j(T_k) for all (k, j)
__global__ void k_planck_table(int nl, int K, const double* __restrict__ nu,
                               const double* __restrict__ Tk, double* __restrict__ Bt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nl * K) return;
  const int k = (int)(i / nl), j = (int)(i % nl);
  Bt[i] = planck_nu(nu[j], Tk[k]);
}

// E_s(T_k) = 4 pi sum_j kabs_s(j) B_j(T_k) dnu_j
__global__ void k_emission(int nl, int S, int K, const double* __restrict__ kabs,
                           const double* __restrict__ Bt, const double* __restrict__ dnu,
                           double* __restrict__ E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * K) return;
  const int s = i / K, k = i % K;
  double e = 0.0;
  for (int j = 0; j < nl; ++j) e += kabs[s * nl + j] * Bt[(int64_t)k * nl + j] * dnu[j];
  E[i] = 4.0 * kPi * e;
}

// Newton weights of the temperature inversion: W[j][s] = 4 pi kabs_s(j) dnu_j
// 2 h nu_j^3 / c^2 and x_j = h nu_j / k
__global__ void k_newton_weights(int nl, int S, const double* __restrict__ kabs,
                                 const double* __restrict__ nu, const double* __restrict__ dnu,
                                 double* __restrict__ W, double* __restrict__ xk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl * S) return;
  const int j = i / S, s = i % S;
  W[i] = 4.0 * kPi * kabs[s * nl + j] * dnu[j] * (2.0 * kH * nu[j] * nu[j] * nu[j] / (kC * kC));
  if (s == 0) xk[j] = kH * nu[j] / kKB;
}

// R_{s,k}(j): normalised running sum over j of kabs_s(j) [B_j(T_{k+1}) - B_j(T_k)] dnu_j
__global__ void k_rows(int nl, int S, int K, const double* __restrict__ kabs,
                       const double* __restrict__ Bt, const double* __restrict__ dnu,
                       double* __restrict__ R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * (K - 1)) return;
  const int s = i / (K - 1), k = i % (K - 1);
  double* row = R + (int64_t)i * nl;
  const double* b0 = Bt + (int64_t)k * nl;
  const double* b1 = Bt + (int64_t)(k + 1) * nl;
  double cum = 0.0;
  for (int j = 0; j < nl; ++j) {
    cum += kabs[s * nl + j] * (b1[j] - b0[j]) * dnu[j];
    row[j] = cum;
  }
  const double inv = cum > 0.0 ? 1.0 / cum : 0.0;
  for (int j = 0; j < nl; ++j) row[j] = cum > 0.0 ? row[j] * inv : 1.0;
  row[nl - 1] = 1.0;
}

// depth and lower corner (finest units) of every leaf: walk each base cube's
// subtree with an explicit stack
__global__ void k_levels(int nb, int L, const int32_t* __restrict__ base_map,
                         const int32_t* __restrict__ nodes, int8_t* __restrict__ level,
                         int4* __restrict__ leaf_lo) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (int64_t)nb * nb * nb) return;
  const int bx = (int)(b % nb), by = (int)((b / nb) % nb), bz = (int)(b / ((int64_t)nb * nb));
  const int32_t e = base_map[b];
  if (e >= 0) {
    level[e] = 0;
    leaf_lo[e] = make_int4(bx << L, by << L, bz << L, 0);
    return;
  }
  int32_t stk_node[16];
  int8_t stk_oct[16];
  int stk_lo[16][3];
  int sp = 0;
  stk_node[0] = -e - 1;
  stk_oct[0] = 0;
  stk_lo[0][0] = bx << L; stk_lo[0][1] = by << L; stk_lo[0][2] = bz << L;
  while (sp >= 0) {
    if (stk_oct[sp] == 8) { --sp; continue; }
    const int o = stk_oct[sp];
    const int32_t c = nodes[(int64_t)stk_node[sp] * 8 + o];
    stk_oct[sp] += 1;
    const int h = 1 << (L - sp - 1);
    const int l0 = stk_lo[sp][0] + (o & 1) * h, l1 = stk_lo[sp][1] + ((o >> 1) & 1) * h,
              l2 = stk_lo[sp][2] + ((o >> 2) & 1) * h;
    if (c >= 0) {
      level[c] = (int8_t)(sp + 1);
      leaf_lo[c] = make_int4(l0, l1, l2, sp + 1);
    } else if (sp + 1 < L && sp + 1 < 16) {
      ++sp;
      stk_node[sp] = -c - 1;
      stk_oct[sp] = 0;
      stk_lo[sp][0] = l0; stk_lo[sp][1] = l1; stk_lo[sp][2] = l2;
    }
  }
}

// grid structure: entries in range, child nodes after their parent (no
// cycles), no node deeper than max_level - 1
__global__ void k_check_grid(int nb, int L, int64_t n_cells, int64_t n_nodes,
                             const int32_t* __restrict__ base_map,
                             const int32_t* __restrict__ nodes, unsigned long long* bad) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (int64_t)nb * nb * nb) return;
  const int32_t e = base_map[b];
  if (e >= 0) { if (e >= n_cells) atomicOr(bad, 16ull); return; }
  if ((int64_t)(-e - 1) >= n_nodes || L < 1) { atomicOr(bad, 16ull); return; }
  int32_t stk_node[16];
  int8_t stk_oct[16];
  int sp = 0;
  stk_node[0] = -e - 1;
  stk_oct[0] = 0;
  while (sp >= 0) {
    if (stk_oct[sp] == 8) { --sp; continue; }
    const int32_t c = nodes[(int64_t)stk_node[sp] * 8 + stk_oct[sp]];
    stk_oct[sp] += 1;
    if (c >= 0) {
      if (c >= n_cells) { atomicOr(bad, 16ull); return; }
    } else {
      const int32_t nd = -c - 1;
      if ((int64_t)nd >= n_nodes || nd <= stk_node[sp] || sp + 2 > L || sp + 1 >= 16) {
        atomicOr(bad, 16ull);
        return;
      }
      ++sp;
      stk_node[sp] = nd;
      stk_oct[sp] = 0;
    }
  }
}

__global__ void k_check_rho(int64_t n_cells, const double* __restrict__ rho,
                            unsigned long long* bad) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  const double r = rho[c];
  if (!(r >= 0.0) || isinf(r)) atomicOr(bad, 1ull);
}

// FP32 density term rho h of a leaf.  A leaf with dust keeps a positive term
// even where rho h is below the smallest normal float (the far wings of a
// disk's vertical profile, tens of scale heights up): rounding it to zero
// would drop the leaf's path-length tally, which counts the path in every
// leaf with dust whatever its density.  The smallest normal float there
// changes no optical depth that FP32 can represent.
__device__ __forceinline__ float rho_h_f32(double r, double h) {
  const float v = (float)(r * h);
  return (r > 0.0 && !(v >= FLT_MIN)) ? FLT_MIN : v;
}

__global__ void k_cells(int64_t n_cells, double h, const double* __restrict__ rho,
                        float* __restrict__ rho_h32) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  rho_h32[c] = rho_h_f32(rho[c], h);
}

// base-map entry packed with the FP32 density term of an unrefined base
// cube, in brick order (4 x 2 x 2 cubes per 128-byte line, binfo_index)
__global__ void k_binfo(int nb, double h, const int32_t* __restrict__ base_map, const double* __restrict__ rho,
                        int2* __restrict__ binfo) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nbase = (int64_t)nb * nb * nb;
  if (b >= nbase) return;
  const int bx = (int)(b % nb), by = (int)((b / nb) % nb), bz = (int)(b / ((int64_t)nb * nb));
  const int32_t e = base_map[b];
  binfo[binfo_index(nb, bx, by, bz)] = make_int2(e, e >= 0 ? __float_as_int(rho_h_f32(rho[e], h)) : 0);
}

__global__ void k_check_species(int nl, int S, const double* __restrict__ lam_um,
                                const double* __restrict__ kabs, const double* __restrict__ ksca,
                                const double* __restrict__ g, unsigned long long* bad) {
  for (int i = threadIdx.x; i < nl * S; i += blockDim.x) {
    const double a = kabs[i], b = ksca[i];
    if (!(a >= 0.0) || !(b >= 0.0) || isinf(a) || isinf(b)) atomicOr(bad, 2ull);
  }
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    if (!(lam_um[j] > 0.0) || (j > 0 && !(lam_um[j] > lam_um[j - 1]))) atomicOr(bad, 4ull);
    if (!(g[j] > -1.0 && g[j] < 1.0)) atomicOr(bad, 8ull);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

Layout make_layout(const mcrt_desc& d) {
  Layout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += (bytes + 255) & ~uint64_t(255);
    return o;
  };
  const uint64_t nl = (uint64_t)d.n_lambda, S = (uint64_t)d.n_species, K = (uint64_t)d.K;
  L.nu = take(8 * nl);
  L.dnu = take(8 * nl);
  L.src_cdf = take(8 * nl);
  L.kext = take(8 * nl);
  L.albedo = take(8 * nl);
  L.gpar = take(8 * nl);
  L.sp_cdf = take(8 * nl * S);
  L.Tk = take(8 * K);
  L.E = take(8 * S * K);
  L.R = take(8 * S * (K - 1) * nl);
  L.Bt = take(8 * K * nl);
  L.Wt = take(8 * nl * S);
  L.xk = take(8 * nl);
  L.kext32 = take(4 * nl);
  L.g32 = take(4 * nl);
  L.rho_h32 = take(4 * (uint64_t)d.n_cells);
  L.level = take((uint64_t)d.n_cells);
  L.leaf_lo = take(16 * (uint64_t)d.n_cells);
  L.binfo = take(8 * binfo_entries(d.nb));
  L.pah_slot = take(4 * S);
  L.scratch = take(sizeof(RunScratch));
  L.total = off;
  return L;
}

hipError_t launch_checks(mcrt_ctx* c, hipStream_t s) {
  const mcrt_desc& d = c->d;
  RunScratch* scr = reinterpret_cast<RunScratch*>(c->tables + c->lay.scratch);
  k_zero_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long*>(scr), (int)(sizeof(RunScratch) / 8));
  k_check_species<<<1, 256, 0, s>>>(d.n_lambda, d.n_species, d.lambda_um, d.kabs, d.ksca, d.g,
                                    &scr->bad_input);
  const int64_t nbase = (int64_t)d.nb * d.nb * d.nb;
  k_check_grid<<<(unsigned)((nbase + 255) / 256), 256, 0, s>>>(d.nb, d.max_level, d.n_cells,
                                                                d.n_nodes, d.base_map, d.nodes,
                                                                &scr->bad_input);
  k_check_rho<<<(unsigned)((d.n_cells + 255) / 256), 256, 0, s>>>(d.n_cells, d.rho, &scr->bad_input);
  return hipGetLastError();
}

hipError_t launch_build_tables(mcrt_ctx* c, hipStream_t s) {
  const mcrt_desc& d = c->d;
  const Layout& L = c->lay;
  unsigned char* T = c->tables;
  auto D = [&](uint64_t o) { return reinterpret_cast<double*>(T + o); };
  auto F = [&](uint64_t o) { return reinterpret_cast<float*>(T + o); };
  const int nl = d.n_lambda, S = d.n_species, K = d.K;
  k_lambda<<<1, 256, 0, s>>>(nl, S, K, d.lambda_um, d.kabs, d.ksca, d.g, d.kind, c->src.teff,
                             d.T_lo, d.T_hi, D(L.nu), D(L.dnu), D(L.src_cdf), D(L.kext),
                             D(L.albedo), D(L.gpar), D(L.sp_cdf), D(L.Tk), F(L.kext32), F(L.g32),
                             reinterpret_cast<int32_t*>(T + L.pah_slot));
  const int64_t nb3 = (int64_t)nl * K;
  k_planck_table<<<(unsigned)((nb3 + 255) / 256), 256, 0, s>>>(nl, K, D(L.nu), D(L.Tk), D(L.Bt));
  k_emission<<<(S * K + 255) / 256, 256, 0, s>>>(nl, S, K, d.kabs, D(L.Bt), D(L.dnu), D(L.E));
  k_rows<<<(S * (K - 1) + 127) / 128, 128, 0, s>>>(nl, S, K, d.kabs, D(L.Bt), D(L.dnu), D(L.R));
  k_newton_weights<<<(nl * S + 255) / 256, 256, 0, s>>>(nl, S, d.kabs, D(L.nu), D(L.dnu), D(L.Wt), D(L.xk));
  const int64_t nbase = (int64_t)d.nb * d.nb * d.nb;
  k_levels<<<(unsigned)((nbase + 255) / 256), 256, 0, s>>>(d.nb, d.max_level, d.base_map, d.nodes,
                                                            reinterpret_cast<int8_t*>(T + L.level),
                                                            reinterpret_cast<int4*>(T + L.leaf_lo));
  k_cells<<<(unsigned)((d.n_cells + 255) / 256), 256, 0, s>>>(d.n_cells, d.base_size, d.rho,
                                                              F(L.rho_h32));
  k_binfo<<<(unsigned)((nbase + 255) / 256), 256, 0, s>>>(d.nb, d.base_size, d.base_map, d.rho,
                                                          reinterpret_cast<int2*>(T + L.binfo));
  return hipGetLastError();
}

}  // namespace mcrt
