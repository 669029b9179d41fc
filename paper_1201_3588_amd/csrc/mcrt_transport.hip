// Packet transport kernel (paper Sec. 2): packets of constant energy are
// followed cell by cell through the cube/subcube grid; an interaction occurs
// where the optical depth along the path reaches the sampled value; scattering
// turns the packet by the Henyey-Greenstein phase function, absorption adds
// the packet to the cell tally and re-emits it isotropically at a frequency
// drawn from the cell temperature before the absorption.
//
// Execution: a persistent pool.  Every lane of a wave64 carries one packet;
// when packets end, the wave refills its dead lanes with new packet ids from a
// global counter (one atomic per wave).  Random numbers come from Philox keyed
// by packet id, so a packet's history does not depend on which lane runs it.
// Geometry runs in R (float or double) on base-cube units, with the current
// cell held as integer finest-level coordinates so face crossings never lose
// the packet; tallies are 64-bit integer atomics.
#include "mcrt_internal.h"

namespace mcrt {

namespace {

template <typename R>
struct TP {
  int nb, L, nl, S, K, n_theta, n_phi, flags, beam_on, trace_cap;
  int64_t n_cells;
  R inv_nf, qscale;
  double h, eps;
  R x0, y0, z0, bx, by, bz;
  uint64_t first_id, n, seed, max_events;
  const int32_t* base_map;
  const int32_t* nodes;
  const double* rho;
  const float* rho_h32;
  const double* kext64;
  const float* kext32;
  const double* albedo;
  const double* gpar;
  const float* g32;
  const double* src_cdf;
  const double* sp_cdf;
  const double* E;
  const double* Rrows;
  const int32_t* kind;
  const int32_t* pah_slot;
  const double* pah_rows;
  const uint64_t* frozen;
  unsigned long long* nabs;
  unsigned long long* sed;
  unsigned long long* jq;
  unsigned long long* counters;
  unsigned long long* work;
  mcrt_trace_rec* trace;
  int32_t* trace_len;
};

__device__ __forceinline__ float rlog(float v) { return logf(v); }
__device__ __forceinline__ double rlog(double v) { return log(v); }
__device__ __forceinline__ float rsqrt0(float v) { return sqrtf(fmaxf(0.0f, v)); }
__device__ __forceinline__ double rsqrt0(double v) { return sqrt(fmax(0.0, v)); }
__device__ __forceinline__ void rsincos(float a, float* s, float* c) { sincosf(a, s, c); }
__device__ __forceinline__ void rsincos(double a, double* s, double* c) { sincos(a, s, c); }
__device__ __forceinline__ float rfloor(float v) { return floorf(v); }
__device__ __forceinline__ double rfloor(double v) { return floor(v); }
__device__ __forceinline__ float rrint(float v) { return rintf(v); }
__device__ __forceinline__ double rrint(double v) { return rint(v); }
__device__ __forceinline__ float ratan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double ratan2(double y, double x) { return atan2(y, x); }

// Henyey-Greenstein (1941) deflection cosine by inverting its CDF
__device__ __forceinline__ double hg_mu(double g, double u) {
  if (fabs(g) < 1e-5) return 2.0 * u - 1.0;
  const double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
  const double mu = (1.0 + g * g - f * f) / (2.0 * g);
  return fmin(1.0, fmax(-1.0, mu));
}

// leaf holding finest-level point F; -1 outside the grid
__device__ __forceinline__ int locate(const int32_t* __restrict__ base_map,
                                      const int32_t* __restrict__ nodes, int nb, int L,
                                      int F0, int F1, int F2, int& lev, int& lo0, int& lo1,
                                      int& lo2) {
  const unsigned ext = (unsigned)nb << L;
  if ((unsigned)F0 >= ext || (unsigned)F1 >= ext || (unsigned)F2 >= ext) return -1;
  int e = base_map[(F0 >> L) + nb * ((F1 >> L) + nb * (F2 >> L))];
  int l = 0;
  while (e < 0) {
    ++l;
    const int sh = L - l;
    const int o = ((F0 >> sh) & 1) | (((F1 >> sh) & 1) << 1) | (((F2 >> sh) & 1) << 2);
    e = nodes[(-e - 1) * 8 + o];
  }
  lev = l;
  const int sh = L - l;
  lo0 = (F0 >> sh) << sh;
  lo1 = (F1 >> sh) << sh;
  lo2 = (F2 >> sh) << sh;
  return e;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), off);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), off);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

template <typename R>
__device__ __forceinline__ void record(const TP<R>& P, uint64_t k, int type, int cell, int j, R x0,
                                       R x1, R x2, R d0, R d1, R d2, R tau) {
  if (!P.trace) return;
  const int n = P.trace_len[k];
  if (n >= P.trace_cap) return;
  mcrt_trace_rec* r = P.trace + (int64_t)k * P.trace_cap + n;
  r->type = type; r->cell = cell; r->j = j; r->pad = 0;
  r->x[0] = x0; r->x[1] = x1; r->x[2] = x2;
  r->d[0] = d0; r->d[1] = d1; r->d[2] = d2;
  r->tau = tau;
  P.trace_len[k] = n + 1;
}

template <typename R>
__device__ __forceinline__ void escape_tally(const TP<R>& P, R d0, R d1, R d2, int j) {
  int bt = (int)rfloor((d2 + R(1)) * R(0.5) * (R)P.n_theta);
  bt = bt < 0 ? 0 : (bt >= P.n_theta ? P.n_theta - 1 : bt);
  R phi = ratan2(d1, d0);
  if (phi < R(0)) phi += R(2.0 * kPi);
  int bp = (int)rfloor(phi / R(2.0 * kPi) * (R)P.n_phi);
  bp = bp < 0 ? 0 : (bp >= P.n_phi ? P.n_phi - 1 : bp);
  atomicAdd(&P.sed[((int64_t)bt * P.n_phi + bp) * P.nl + j], 1ull);
}

template <typename R>
__global__ void __launch_bounds__(256) k_transport(const TP<R> P) {
  extern __shared__ double smem[];
  double* s_alb = smem;
  double* s_src = s_alb + P.nl;
  R* s_kext = reinterpret_cast<R*>(s_src + P.nl);
  for (int j = threadIdx.x; j < P.nl; j += blockDim.x) {
    s_alb[j] = P.albedo[j];
    s_src[j] = P.src_cdf[j];
    s_kext[j] = sizeof(R) == 8 ? (R)P.kext64[j] : (R)P.kext32[j];
  }
  __syncthreads();

  const bool f64 = sizeof(R) == 8;
  const int lane = __lane_id();
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  const int L = P.L;
  const R inv_nf = P.inv_nf;
  const uint32_t key0 = (uint32_t)P.seed, key1 = (uint32_t)(P.seed >> 32);
  const bool tally_j = (P.flags & MCRT_FLAG_TALLY_J) && P.jq != nullptr;

  bool alive = false, exhausted = false;
  uint64_t pid = 0, kidx = 0;
  uint64_t events = 0;
  R x0 = 0, x1 = 0, x2 = 0, d0 = 0, d1 = 0, d2 = 1, tau = 0;
  int j = 0, cell = 0, lev = 0, lo0 = 0, lo1 = 0, lo2 = 0;
  unsigned long long c_launch = 0, c_esc = 0, c_kill = 0, c_term = 0, c_scat = 0, c_abs = 0,
                     c_cross = 0, c_tlo = 0, c_thi = 0, c_pah = 0, c_zero = 0, c_jseg = 0;

  for (;;) {
    if (!exhausted) {
      const unsigned long long dead = __ballot(!alive);
      if (dead) {
        const int nd = __popcll(dead);
        const int leader = __ffsll((long long)dead) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(P.work, (unsigned long long)nd);
        base = __shfl(base, leader);
        if (base + (unsigned long long)nd >= P.n) exhausted = true;
        if (!alive) {
          const uint64_t k = base + (uint64_t)__popcll(dead & lt_mask);
          if (k < P.n) {
            // launch (event slot 0): bin from the source CDF, direction, optical depth
            kidx = k;
            pid = P.first_id + k;
            events = 0;
            uint32_t w[4];
            philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), 0u, 0u, key0, key1, w);
            j = cdf_search(s_src, P.nl, u24(w[0]));
            if (P.beam_on) { d0 = P.bx; d1 = P.by; d2 = P.bz; }
            else {
              const R mu = (R)(2.0 * u24(w[1]) - 1.0);
              const R st = rsqrt0(R(1) - mu * mu);
              R sp, cp;
              rsincos((R)(2.0 * kPi * u24(w[2])), &sp, &cp);
              d0 = st * cp; d1 = st * sp; d2 = mu;
            }
            tau = -rlog((R)u24(w[3]));
            x0 = P.x0; x1 = P.y0; x2 = P.z0;
            const R nf = (R)(1 << L);
            cell = locate(P.base_map, P.nodes, P.nb, L, (int)rfloor(x0 * nf), (int)rfloor(x1 * nf),
                          (int)rfloor(x2 * nf), lev, lo0, lo1, lo2);
            c_launch++;
            record(P, kidx, 0, cell, j, x0, x1, x2, d0, d1, d2, tau);
            if (cell < 0) {
              c_esc++;
              escape_tally(P, d0, d1, d2, j);
              record(P, kidx, 4, -1, j, x0, x1, x2, d0, d1, d2, tau);
            } else {
              alive = true;
            }
          }
        }
      }
    }
    if (!__any(alive)) {
      if (exhausted) break;
      continue;
    }
    if (!alive) continue;

    // ---- one segment: exit distance from the current leaf (lowest axis wins ties)
    const int span = 1 << (L - lev);
    const R side = (R)span * inv_nf;
    R tex = (R)INFINITY;
    int ax = -1;
    {
      const R b0 = (R)lo0 * inv_nf, b1 = (R)lo1 * inv_nf, b2 = (R)lo2 * inv_nf;
      R t;
      if (d0 != R(0)) {
        t = d0 > R(0) ? (b0 + side - x0) / d0 : (b0 - x0) / d0;
        t = t < R(0) ? R(0) : t;
        if (t < tex) { tex = t; ax = 0; }
      }
      if (d1 != R(0)) {
        t = d1 > R(0) ? (b1 + side - x1) / d1 : (b1 - x1) / d1;
        t = t < R(0) ? R(0) : t;
        if (t < tex) { tex = t; ax = 1; }
      }
      if (d2 != R(0)) {
        t = d2 > R(0) ? (b2 + side - x2) / d2 : (b2 - x2) / d2;
        t = t < R(0) ? R(0) : t;
        if (t < tex) { tex = t; ax = 2; }
      }
    }
    R alpha;
    bool dusty;
    if (f64) {
      const double r = P.rho[cell];
      alpha = (R)(r * (double)s_kext[j] * P.h);
      dusty = r > 0.0;
    } else {
      const float r = P.rho_h32[cell];
      alpha = (R)(r * (float)s_kext[j]);
      dusty = r > 0.0f;
    }

    if (alpha > R(0) && tau < alpha * tex) {
      // ---- interaction inside this cell
      const R s = tau / alpha;
      x0 += s * d0; x1 += s * d1; x2 += s * d2;
      if (tally_j && dusty) {
        atomicAdd(&P.jq[(int64_t)j * P.n_cells + cell], (unsigned long long)rrint(s * P.qscale));
        c_jseg++;
      }
      events += 1;
      if (events > P.max_events) {
        c_kill++;
        alive = false;
        record(P, kidx, 5, cell, j, x0, x1, x2, d0, d1, d2, tau);
        continue;
      }
      uint32_t w[4], v[4];
      philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), (uint32_t)events, 0u, key0, key1, w);
      philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), (uint32_t)events, 1u, key0, key1, v);
      const double phi = 2.0 * kPi * u24(w[2]);
      R sp, cp;
      rsincos((R)phi, &sp, &cp);
      if (u24(w[0]) <= s_alb[j]) {
        // scattering: new direction from the phase function
        const R mu = (R)hg_mu(P.gpar[j], u24(w[1]));
        const R st = rsqrt0(R(1) - mu * mu);
        if (d2 > R(0.99999) || d2 < R(-0.99999)) {
          d0 = st * cp; d1 = st * sp; d2 = d2 >= R(0) ? mu : -mu;
        } else {
          const R tmp = rsqrt0(R(1) - d2 * d2);
          const R n0 = st * (d0 * d2 * cp - d1 * sp) / tmp + d0 * mu;
          const R n1 = st * (d1 * d2 * cp + d0 * sp) / tmp + d1 * mu;
          const R n2 = -st * cp * tmp + d2 * mu;
          d0 = n0; d1 = n1; d2 = n2;
        }
        c_scat++;
        tau = -rlog((R)u24(w[3]));
        record(P, kidx, 2, cell, j, x0, x1, x2, d0, d1, d2, tau);
      } else {
        // absorption: species, tally, new frequency, isotropic re-emission
        const int sp_i = cdf_search(P.sp_cdf + (int64_t)j * P.S, P.S, u24(w[1]));
        unsigned long long before = atomicAdd(&P.nabs[(int64_t)cell * P.S + sp_i], 1ull);
        c_abs++;
        if (P.flags & MCRT_FLAG_FROZEN_T) before = P.frozen[(int64_t)cell * P.S + sp_i];
        if (P.flags & MCRT_FLAG_KILL_ON_ABSORB) {
          c_term++;
          alive = false;
          record(P, kidx, 3, cell, j, x0, x1, x2, d0, d1, d2, tau);
          continue;
        }
        if (P.kind[sp_i] == 0) {
          const double vol = pow(P.h * ldexp(1.0, -lev), 3.0);
          const double pw = (double)before * P.eps / (P.rho[cell] * vol);
          const double* E = P.E + (int64_t)sp_i * P.K;
          int kb;
          if (pw < E[0]) {
            kb = 0;
            c_tlo++;
          } else {
            int a = 0, b = P.K - 1;
            if (E[P.K - 1] <= pw) a = P.K - 1;
            else
              while (b - a > 1) {
                const int m = (a + b) >> 1;
                if (E[m] <= pw) a = m; else b = m;
              }
            kb = a;
            if (kb > P.K - 2) { kb = P.K - 2; c_thi++; }
          }
          j = cdf_search(P.Rrows + ((int64_t)sp_i * (P.K - 1) + kb) * P.nl, P.nl, u24(v[0]));
        } else {
          const double* row = P.pah_rows + ((int64_t)P.pah_slot[sp_i] * P.n_cells + cell) * P.nl;
          j = cdf_search(row, P.nl, u24(v[0]));
          c_pah++;
        }
        const R mu = (R)(2.0 * u24(v[1]) - 1.0);
        const R st = rsqrt0(R(1) - mu * mu);
        d0 = st * cp; d1 = st * sp; d2 = mu;
        tau = -rlog((R)u24(w[3]));
        record(P, kidx, 3, cell, j, x0, x1, x2, d0, d1, d2, tau);
      }
      continue;
    }

    // ---- cross the face into the neighbour
    if (alpha > R(0)) tau -= alpha * tex;
    if (tally_j && dusty) {
      atomicAdd(&P.jq[(int64_t)j * P.n_cells + cell], (unsigned long long)rrint(tex * P.qscale));
      c_jseg++;
    }
    c_cross++;
    if (tex == R(0)) c_zero++;
    x0 += tex * d0; x1 += tex * d1; x2 += tex * d2;
    const R nf = (R)(1 << L);
    int G0, G1, G2;
    {
      const int f0 = (int)rfloor(x0 * nf), f1 = (int)rfloor(x1 * nf), f2 = (int)rfloor(x2 * nf);
      G0 = f0 < lo0 ? lo0 : (f0 > lo0 + span - 1 ? lo0 + span - 1 : f0);
      G1 = f1 < lo1 ? lo1 : (f1 > lo1 + span - 1 ? lo1 + span - 1 : f1);
      G2 = f2 < lo2 ? lo2 : (f2 > lo2 + span - 1 ? lo2 + span - 1 : f2);
    }
    if (ax == 0) {
      const int face = d0 > R(0) ? lo0 + span : lo0;
      x0 = (R)face * inv_nf;
      G0 = d0 > R(0) ? lo0 + span : lo0 - 1;
    } else if (ax == 1) {
      const int face = d1 > R(0) ? lo1 + span : lo1;
      x1 = (R)face * inv_nf;
      G1 = d1 > R(0) ? lo1 + span : lo1 - 1;
    } else {
      const int face = d2 > R(0) ? lo2 + span : lo2;
      x2 = (R)face * inv_nf;
      G2 = d2 > R(0) ? lo2 + span : lo2 - 1;
    }
    cell = locate(P.base_map, P.nodes, P.nb, L, G0, G1, G2, lev, lo0, lo1, lo2);
    if (cell < 0) {
      c_esc++;
      alive = false;
      escape_tally(P, d0, d1, d2, j);
      record(P, kidx, 4, -1, j, x0, x1, x2, d0, d1, d2, tau);
    } else {
      record(P, kidx, 1, cell, j, x0, x1, x2, d0, d1, d2, tau);
    }
  }

  // ---- counters: one atomic per wave per slot
  unsigned long long vals[12] = {c_launch, c_esc, c_kill, c_term, c_scat, c_abs,
                                 c_cross, c_tlo, c_thi, c_pah, c_zero, c_jseg};
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const unsigned long long s = wave_sum(vals[i]);
    if (lane == 0 && s) atomicAdd(&P.counters[i], s);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

template <typename R>
hipError_t launch_t(mcrt_ctx* c, uint64_t first_id, uint64_t n, const mcrt_run_opts& o,
                    const mcrt_tallies& t, hipStream_t s) {
  const mcrt_desc& d = c->d;
  const Layout& L = c->lay;
  unsigned char* T = c->tables;
  TP<R> P{};
  P.nb = d.nb; P.L = d.max_level; P.nl = d.n_lambda; P.S = d.n_species; P.K = d.K;
  P.n_theta = d.n_theta; P.n_phi = d.n_phi; P.flags = o.flags;
  P.beam_on = c->src.beam_on; P.trace_cap = o.trace_cap;
  P.n_cells = d.n_cells;
  P.inv_nf = (R)ldexp(1.0, -d.max_level);
  P.qscale = (R)ldexp(1.0, d.max_level + 16);
  P.h = d.base_size;
  P.eps = c->src.lum / (double)o.n_total;
  P.x0 = (R)((c->src.pos[0] - d.box_min[0]) / d.base_size);
  P.y0 = (R)((c->src.pos[1] - d.box_min[1]) / d.base_size);
  P.z0 = (R)((c->src.pos[2] - d.box_min[2]) / d.base_size);
  P.bx = (R)c->src.beam[0]; P.by = (R)c->src.beam[1]; P.bz = (R)c->src.beam[2];
  P.first_id = first_id; P.n = n; P.seed = o.seed; P.max_events = o.max_events;
  P.base_map = d.base_map; P.nodes = d.nodes; P.rho = d.rho;
  P.rho_h32 = reinterpret_cast<const float*>(T + L.rho_h32);
  P.kext64 = reinterpret_cast<const double*>(T + L.kext);
  P.kext32 = reinterpret_cast<const float*>(T + L.kext32);
  P.albedo = reinterpret_cast<const double*>(T + L.albedo);
  P.gpar = reinterpret_cast<const double*>(T + L.gpar);
  P.g32 = reinterpret_cast<const float*>(T + L.g32);
  P.src_cdf = reinterpret_cast<const double*>(T + L.src_cdf);
  P.sp_cdf = reinterpret_cast<const double*>(T + L.sp_cdf);
  P.E = reinterpret_cast<const double*>(T + L.E);
  P.Rrows = reinterpret_cast<const double*>(T + L.R);
  P.kind = d.kind;
  P.pah_slot = reinterpret_cast<const int32_t*>(T + L.pah_slot);
  P.pah_rows = o.pah_rows;
  P.frozen = o.frozen_nabs;
  P.nabs = reinterpret_cast<unsigned long long*>(t.nabs);
  P.sed = reinterpret_cast<unsigned long long*>(t.sed);
  P.jq = reinterpret_cast<unsigned long long*>(t.jq);
  P.counters = reinterpret_cast<unsigned long long*>(t.counters);
  RunScratch* scr = reinterpret_cast<RunScratch*>(T + L.scratch);
  P.work = &scr->work_counter;
  P.trace = o.trace;
  P.trace_len = o.trace_len;
  k_zero_u64<<<1, 64, 0, s>>>(&scr->work_counter, 1);
  const uint64_t want = (n + 255) / 256;
  uint64_t blocks = o.grid_blocks > 0 ? (uint64_t)o.grid_blocks : (uint64_t)c->n_cu * 8;
  if (blocks > want) blocks = want;
  if (blocks < 1) blocks = 1;
  const size_t lds = (size_t)d.n_lambda * (2 * sizeof(double) + sizeof(R));
  k_transport<R><<<(unsigned)blocks, 256, lds, s>>>(P);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_transport(mcrt_ctx* c, uint64_t first_id, uint64_t n, const mcrt_run_opts& o,
                            const mcrt_tallies& t, hipStream_t s) {
  if (c->d.precision == MCRT_F64) return launch_t<double>(c, first_id, n, o, t, s);
  return launch_t<float>(c, first_id, n, o, t, s);
}

}  // namespace mcrt
