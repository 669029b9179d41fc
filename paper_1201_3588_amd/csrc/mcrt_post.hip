// After a pass: equilibrium temperatures (FP64) from the absorbed-packet
// tallies (paper Sec. 2: each absorption raises the cell energy by eps and
// thereby its temperature) and the path-length mean intensity J_nu per cell
// (Lucy 1999, the packet scheme the method goes back to).
#include "mcrt_internal.h"

namespace mcrt {

namespace {

// One thread per (cell, species): solve N eps = rho V E_s(T).  The bracket
// [T_k, T_{k+1}] comes from the tabulated E_s(T_k); inside it a safeguarded
// Newton iteration runs on the exact bin sum
//   E_s(T) = sum_j W[j][s] / expm1(x_j / T),  W = 4 pi kabs_s(j) dnu_j 2 h nu_j^3 / c^2,
// x_j = h nu_j / k.  Newton converges quadratically from the power-law start
// inside the bracket, so a step below 1e-8 T leaves an error far below FP64
// resolution and ends the iteration.  W and x are staged in LDS when they fit.
__global__ void __launch_bounds__(256) k_temperatures(
    int64_t n_cells, int S, int nl, int K, double h, double eps, double T_lo, double T_hi,
    const int32_t* __restrict__ kind, const double* __restrict__ Wg, const double* __restrict__ xg,
    const double* __restrict__ Tk, const double* __restrict__ E, const double* __restrict__ rho,
    const int8_t* __restrict__ level, const unsigned long long* __restrict__ nabs,
    double* __restrict__ T, int use_lds) {
  extern __shared__ double sm[];
  const double* W = Wg;
  const double* xk = xg;
  if (use_lds) {
    double* sW = sm;
    double* sx = sm + (int64_t)nl * S;
    for (int i = threadIdx.x; i < nl * S; i += blockDim.x) sW[i] = Wg[i];
    for (int i = threadIdx.x; i < nl; i += blockDim.x) sx[i] = xg[i];
    __syncthreads();
    W = sW;
    xk = sx;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cells * S) return;
  const int64_t c = i / S;
  const int s = (int)(i % S);
  if (kind[s] != 0) { T[i] = 0.0; return; }
  const unsigned long long N = nabs[i];
  const double r = rho[c];
  if (N == 0ull || !(r > 0.0)) { T[i] = T_lo; return; }
  const double vol = ldexp(h * h * h, -3 * (int)level[c]);
  const double p = (double)N * eps / (r * vol);
  const double* Es = E + (int64_t)s * K;
  if (p <= Es[0]) { T[i] = T_lo; return; }
  if (p >= Es[K - 1]) { T[i] = T_hi; return; }
  int a = 0, b = K - 1;                // Es[a] <= p < Es[b]
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if (Es[m] <= p) a = m; else b = m;
  }
  double lo = Tk[a], hi = Tk[b];
  // starting point: the table index as a cubic in ln E through the four
  // nearest table points (ln T is linear in the index), so that one exact
  // evaluation usually converges
  double t;
  {
    const int k0 = a - 1 < 0 ? 0 : (a + 2 > K - 1 ? K - 4 : a - 1);
    const double y = log(p);
    double kk = 0.0;
    if (K >= 4) {
      double ys[4];
      for (int q = 0; q < 4; ++q) ys[q] = log(Es[k0 + q]);
      for (int q = 0; q < 4; ++q) {
        double l = 1.0;
        for (int r = 0; r < 4; ++r)
          if (r != q) l *= (y - ys[r]) / (ys[q] - ys[r]);
        kk += l * (double)(k0 + q);
      }
    }
    t = (K >= 4 && kk >= (double)a && kk <= (double)b)
            ? Tk[0] * exp(log(Tk[K - 1] / Tk[0]) * kk / (double)(K - 1))
            : lo * exp(log(hi / lo) * (log(p / Es[a]) / log(Es[b] / Es[a])));
  }
  for (int it = 0; it < 40; ++it) {
    const double it_ = 1.0 / t;
    double e = 0.0, de = 0.0;
    for (int j = 0; j < nl; ++j) {
      const double x = xk[j] * it_;
      const double em1 = expm1(x);
      const double q = 1.0 / em1;          // 0 once expm1 overflows
      const double w = W[(int64_t)j * S + s];
      e += w * q;
      de += w * x * q * (1.0 + q);
    }
    de *= it_;
    const double f = e - p;
    if (f > 0.0) hi = t; else lo = t;
    double tn = de > 0.0 ? t - f / de : 0.5 * (lo + hi);
    if (!(tn >= lo && tn <= hi)) tn = 0.5 * (lo + hi);   // a converged step may land on an end
    const double step = fabs(tn - t);
    t = tn;
    if (step <= 1e-8 * t || hi - lo <= 1e-15 * hi) break;
  }
  T[i] = t;
}

// J[c][j] = eps dq Q[j][c] / (4 pi V_c dnu_j): 32x32 tiles through LDS turn
// the [lambda][cell] tally into the [cell][lambda] field.
__global__ void k_mean_intensity(int64_t n_cells, int nl, double h, int L, double eps,
                                 const double* __restrict__ dnu, const int8_t* __restrict__ level,
                                 const unsigned long long* __restrict__ jq, float* __restrict__ J) {
  __shared__ double tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32;
  const int j0 = blockIdx.y * 32;
  const double dq = h * ldexp(1.0, -(L + 16));
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int j = j0 + r;
    const int64_t c = c0 + threadIdx.x;
    if (j < nl && c < n_cells) tile[r][threadIdx.x] = (double)jq[(int64_t)j * n_cells + c];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int64_t c = c0 + r;
    const int j = j0 + threadIdx.x;
    if (j < nl && c < n_cells) {
      const double vol = ldexp(h * h * h, -3 * (int)level[c]);
      J[c * nl + j] = (float)(eps * dq * tile[threadIdx.x][r] / (4.0 * kPi * vol * dnu[j]));
    }
  }
}

__global__ void k_thin_field(int64_t n_cells, int nl, double h, int L, double bx, double by, double bz,
                             double sx, double sy, double sz, double lum,
                             const double* __restrict__ src_cdf, const double* __restrict__ dnu,
                             const int4* __restrict__ leaf_lo, float* __restrict__ J) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cells * nl) return;
  const int64_t c = i / nl;
  const int j = (int)(i % nl);
  const int4 lo = leaf_lo[c];
  const double fine = h * ldexp(1.0, -L);
  const double span = ldexp(1.0, L - lo.w);
  const double dx = bx + ((double)lo.x + 0.5 * span) * fine - sx;
  const double dy = by + ((double)lo.y + 0.5 * span) * fine - sy;
  const double dz = bz + ((double)lo.z + 0.5 * span) * fine - sz;
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double half = 0.5 * span * fine;
  if (r < half) r = half;
  const double w = src_cdf[j] - (j > 0 ? src_cdf[j - 1] : 0.0);
  J[i] = (float)(lum * w / (16.0 * kPi * kPi * r * r * dnu[j]));
}

// mass of dust per leaf: rho_c h^3 2^(-3 level_c)
__global__ void k_cell_mass(int64_t n_cells, double h3, const double* __restrict__ rho,
                            const int8_t* __restrict__ level, double* __restrict__ mass) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  mass[c] = rho[c] * ldexp(h3, -3 * (int)level[c]);
}

}  // namespace

hipError_t launch_cell_mass(mcrt_ctx* c, double* mass, hipStream_t s) {
  const mcrt_desc& d = c->d;
  const double h3 = d.base_size * d.base_size * d.base_size;
  k_cell_mass<<<(unsigned)((d.n_cells + 255) / 256), 256, 0, s>>>(
      d.n_cells, h3, d.rho, reinterpret_cast<const int8_t*>(c->tables + c->lay.level), mass);
  return hipGetLastError();
}

hipError_t launch_thin_field(mcrt_ctx* c, float* J, hipStream_t s) {
  const mcrt_desc& d = c->d;
  const Layout& L = c->lay;
  unsigned char* B = c->tables;
  const int64_t n = d.n_cells * d.n_lambda;
  k_thin_field<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
      d.n_cells, d.n_lambda, d.base_size, d.max_level, d.box_min[0], d.box_min[1], d.box_min[2],
      c->src.pos[0], c->src.pos[1], c->src.pos[2], c->src.lum,
      reinterpret_cast<const double*>(B + L.src_cdf), reinterpret_cast<const double*>(B + L.dnu),
      reinterpret_cast<const int4*>(B + L.leaf_lo), J);
  return hipGetLastError();
}

hipError_t launch_temperatures(mcrt_ctx* c, const uint64_t* nabs, uint64_t n_total, double* T,
                               hipStream_t s) {
  const mcrt_desc& d = c->d;
  const Layout& L = c->lay;
  unsigned char* B = c->tables;
  const int64_t n = d.n_cells * d.n_species;
  const size_t lds = sizeof(double) * ((size_t)d.n_lambda * d.n_species + d.n_lambda);
  const int use_lds = lds <= 48 * 1024;
  k_temperatures<<<(unsigned)((n + 255) / 256), 256, use_lds ? lds : 0, s>>>(
      d.n_cells, d.n_species, d.n_lambda, d.K, d.base_size, c->src.lum / (double)n_total, d.T_lo,
      d.T_hi, d.kind, reinterpret_cast<const double*>(B + L.Wt), reinterpret_cast<const double*>(B + L.xk),
      reinterpret_cast<const double*>(B + L.Tk), reinterpret_cast<const double*>(B + L.E), d.rho,
      reinterpret_cast<const int8_t*>(B + L.level), reinterpret_cast<const unsigned long long*>(nabs),
      T, use_lds);
  return hipGetLastError();
}

hipError_t launch_mean_intensity(mcrt_ctx* c, const uint64_t* jq, uint64_t n_total, float* J,
                                 hipStream_t s) {
  const mcrt_desc& d = c->d;
  const Layout& L = c->lay;
  unsigned char* B = c->tables;
  dim3 grid((unsigned)((d.n_cells + 31) / 32), (unsigned)((d.n_lambda + 31) / 32));
  dim3 block(32, 8);
  k_mean_intensity<<<grid, block, 0, s>>>(d.n_cells, d.n_lambda, d.base_size, d.max_level,
                                          c->src.lum / (double)n_total,
                                          reinterpret_cast<const double*>(B + L.dnu),
                                          reinterpret_cast<const int8_t*>(B + L.level),
                                          reinterpret_cast<const unsigned long long*>(jq), J);
  return hipGetLastError();
}

}  // namespace mcrt
