// Packet transport kernel (paper Sec. 2): packets of constant energy are
// followed cell by cell through the cube/subcube grid; an interaction occurs
// where the optical depth along the path reaches the sampled value; scattering
// turns the packet by the Henyey-Greenstein phase function, absorption adds
// the packet to the cell tally and re-emits it isotropically at a frequency
// drawn from the cell temperature before the absorption.
//
// Execution: a persistent pool.  Every lane of a wave64 carries one packet and
// marches it cell after cell; when packets end, the wave refills its dead
// lanes with new packet ids from a global counter (one atomic per wave).
// Random numbers come from Philox keyed by packet id, so a packet's history
// does not depend on which lane runs it.  Geometry runs in R (float or double)
// on base-cube units, with the current cell held as integer finest-level
// coordinates so face crossings never lose the packet; tallies are 64-bit
// integer sums (atomics, or for the path tally records added after the
// kernel).
#include "mcrt_internal.h"

namespace mcrt {

namespace {

template <typename R>
struct TP {
  int nb, L, nl, S, K, n_theta, n_phi, flags, beam_on, trace_cap;
  int64_t n_cells;
  R inv_nf, qscale;
  double h, h3, eps;
  double x0, y0, z0;
  R bx, by, bz;
  uint64_t first_id, n, seed, max_events;
  const int32_t* base_map;
  const int2* binfo;          // FP32: {base_map entry, float bits of rho*h}
  const int32_t* nodes;
  const double* rho;
  const float* rho_h32;
  const double* kext64;
  const float* kext32;
  const double* albedo;
  const double* gpar;
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
  ImgP img;
  // next-event images: record queue, its capacity and fill counter, leaf
  // tables for restarting a march from a record, and the images
  unsigned char* peel_q;
  uint64_t peel_cap;
  unsigned long long* peel_count;
  const int8_t* level;
  const int4* leaf_lo;
  unsigned long long* peel;
  unsigned long long* peel_sed;     // [n_obs][nl] or null: every event is queued
  // deferred path tally: record buffer, its capacity and fill counter
  unsigned long long* jrec;
  uint64_t jrec_cap;
  unsigned long long* jrec_count;
};

// The kernel's argument block, read through an address the compiler cannot
// see through: in the launch and interaction branches the fields are loaded
// (scalar loads from the argument segment) where they are used, instead of
// being held in scalar registers across the whole march, where they would
// crowd out (and spill) the values the march itself uses.
template <typename R>
using ArgPtr = const __attribute__((address_space(4))) TP<R>*;
template <typename R>
__device__ __forceinline__ ArgPtr<R> cold_args() {
  ArgPtr<R> q = (ArgPtr<R>)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(q));
  return q;
}

// One queued next-event: where (base-cube units, inside leaf `cell`), in which
// bin, and for a scattering the direction the packet arrived along.
struct PeelRec {
  double x[3];
  double din[3];
  int32_t cell, j, type, pad;     // type 0: isotropic emission, 1: scattering
};
static_assert(sizeof(PeelRec) == MCRT_PEEL_REC_BYTES, "peel record size");

__device__ __forceinline__ float rlog(float v) { return logf(v); }
__device__ __forceinline__ double rlog(double v) { return log(v); }
__device__ __forceinline__ float rsqrt0(float v) { return sqrtf(fmaxf(0.0f, v)); }
__device__ __forceinline__ double rsqrt0(double v) { return sqrt(fmax(0.0, v)); }
// sin and cos of 2 pi u for u in (0, 1]: FP32 uses the hardware sine/cosine,
// whose argument is in revolutions (no range reduction needed here); FP64
// uses the library sincos.
__device__ __forceinline__ void sincos_rev(double u, float* s, float* c) {
  float r = (float)u;
  r = r > 0.5f ? r - 1.0f : r;            // exact: u is a multiple of 2^-24
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sincos_rev(double u, double* s, double* c) {
  sincos(2.0 * kPi * u, s, c);
}
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

// Leaf holding finest-level point F (-1 outside the grid) and its density
// term: rho*h (FP32 path, packed with the base-map entry for unrefined base
// cubes so the common case is one 8-byte load) or rho (FP64 path).
template <typename R>
__device__ __forceinline__ int locate(const TP<R>& P, int F0, int F1, int F2, int& lev, int& lo0,
                                      int& lo1, int& lo2, R& dens) {
  const int L = P.L, nb = P.nb;
  const unsigned ext = (unsigned)nb << L;
  if ((unsigned)F0 >= ext || (unsigned)F1 >= ext || (unsigned)F2 >= ext) return -1;
  int e;
  if (sizeof(R) == 4) {
    // one 8-byte load, both halves materialised at once (otherwise the
    // compiler defers the density half past the refined-cube test, a second
    // dependent load per crossing)
    uint64_t raw = *reinterpret_cast<const uint64_t*>(P.binfo + binfo_index(nb, F0 >> L, F1 >> L, F2 >> L));
    asm volatile("" : "+v"(raw));
    e = (int)(uint32_t)raw;
    dens = (R)__uint_as_float((uint32_t)(raw >> 32));
  } else {
    e = P.base_map[(F0 >> L) + nb * ((F1 >> L) + nb * (F2 >> L))];
  }
  int l = 0;
  if (e < 0) {
    do {
      ++l;
      const int sh = L - l;
      const int o = ((F0 >> sh) & 1) | (((F1 >> sh) & 1) << 1) | (((F2 >> sh) & 1) << 2);
      e = P.nodes[(-e - 1) * 8 + o];
    } while (e < 0);
    if (sizeof(R) == 4) dens = (R)P.rho_h32[e];
  }
  if (sizeof(R) == 8) dens = (R)P.rho[e];
  lev = l;
  const int sh = L - l;
  lo0 = (F0 >> sh) << sh;
  lo1 = (F1 >> sh) << sh;
  lo2 = (F2 >> sh) << sh;
  return e;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = (uint32_t)__shfl_xor((int)v, off);
    v = o > v ? o : v;
  }
  return v;
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
__device__ __forceinline__ void record(const TP<R>& P, uint64_t k, int type, int cell, int j,
                                       double x0, double x1, double x2, R d0, R d1, R d2, R tau) {
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
__device__ __forceinline__ void escape_tally(R d0, R d1, R d2, int j) {
  const ArgPtr<R> Q = cold_args<R>();
  int bt = (int)rfloor((d2 + R(1)) * R(0.5) * (R)Q->n_theta);
  bt = bt < 0 ? 0 : (bt >= Q->n_theta ? Q->n_theta - 1 : bt);
  R phi = ratan2(d1, d0);
  if (phi < R(0)) phi += R(2.0 * kPi);
  int bp = (int)rfloor(phi / R(2.0 * kPi) * (R)Q->n_phi);
  bp = bp < 0 ? 0 : (bp >= Q->n_phi ? Q->n_phi - 1 : bp);
  atomicAdd(&Q->sed[((int64_t)bt * Q->n_phi + bp) * Q->nl + j], 1ull);
}

// escape images: the exit point x (base-cube units), moved back along the ray
// to the observer's image plane, in plane pixels (see mcrt_observers)
template <typename R>
__device__ __forceinline__ void image_tally(double x0, double x1, double x2, R d0, R d1, R d2, int j) {
  const ArgPtr<R> Q = cold_args<R>();
  const __attribute__((address_space(4))) ImgP& I = Q->img;
  int l = -1;
  for (int q = 0; q < I.n_l; ++q)
    if (I.lsel[q] == j) l = q;
  if (l < 0) return;
  const double X0 = I.off[0] + x0 * I.h, X1 = I.off[1] + x1 * I.h, X2 = I.off[2] + x2 * I.h;
  const double e0 = d0, e1 = d1, e2 = d2;
  for (int o = 0; o < I.n_obs; ++o) {
    const auto* n = I.n[o];
    const double dn = e0 * n[0] + e1 * n[1] + e2 * n[2];
    if (dn < I.cos_cone) continue;
    const double t = (X0 * n[0] + X1 * n[1] + X2 * n[2]) / dn;
    const double p0 = X0 - t * e0, p1 = X1 - t * e1, p2 = X2 - t * e2;
    const double a = p0 * I.e1[o][0] + p1 * I.e1[o][1] + p2 * I.e1[o][2];
    const double b = p0 * I.e2[o][0] + p1 * I.e2[o][1] + p2 * I.e2[o][2];
    const double fx = floor((a + I.w) / (2.0 * I.w) * I.npix), fy = floor((b + I.w) / (2.0 * I.w) * I.npix);
    if (fx < 0.0 || fy < 0.0 || fx >= I.npix || fy >= I.npix) continue;
    atomicAdd(&I.image[(((int64_t)o * I.n_l + l) * I.npix + (int64_t)fy) * I.npix + (int64_t)fx], 1ull);
  }
}

// Queues a next-event record when bin j is imaged (rare: a few imaged bins
// out of the whole grid), or for every event when the observers' SEDs are
// on; records past the capacity are dropped and counted by the march kernel.
template <typename R>
__device__ __forceinline__ void peel_push(double x0, double x1, double x2, int cell, int j, int type, R d0, R d1,
                                          R d2) {
  const ArgPtr<R> Q = cold_args<R>();
  bool imaged = Q->peel_sed != nullptr;
  for (int q = 0; q < Q->img.n_l; ++q) imaged |= Q->img.lsel[q] == j;
  if (!imaged) return;
  const unsigned long long k = atomicAdd(Q->peel_count, 1ull);
  if (k >= Q->peel_cap) return;
  PeelRec* r = reinterpret_cast<PeelRec*>(Q->peel_q) + k;
  r->x[0] = x0; r->x[1] = x1; r->x[2] = x2;
  r->din[0] = (double)d0; r->din[1] = (double)d1; r->din[2] = (double)d2;
  r->cell = cell; r->j = j; r->type = type; r->pad = 0;
}

// Deferred path tally: records staged per wave in LDS (kStage per wave)
// and copied to the wave's chunk of the record buffer in bulk.  A wave's
// march stops when its staging area could not take another wave of records:
// 768 rather than 512 lets it run longer (1.4 % on the 256^3 disk), and five
// blocks of four waves still fit a CU's LDS.
constexpr uint32_t kStage = 768;

// Copies the wave's n staged records to the record buffer: contiguous
// positions in the wave's current chunk [rcur, rcur + rleft), claiming
// chunks of kRecChunk records as needed; once the buffer is exhausted (rfull)
// the records go to the tally by atomic add (the tally is the same).  Every
// lane of the wave calls it with the same (wave-uniform) arguments.
template <typename R>
__device__ __forceinline__ void flush_records(const unsigned long long* rec, uint32_t n, uint64_t& rcur,
                                              uint64_t& rleft, bool& rfull) {
  const ArgPtr<R> Q = cold_args<R>();
  const int lane = __lane_id();
  uint32_t done = 0;
  while (done < n) {
    if (!rfull && rleft == 0) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(Q->jrec_count, (unsigned long long)kRecChunk);
      base = __shfl(base, 0);
      if (base + kRecChunk <= Q->jrec_cap) {
        rcur = base;
        rleft = kRecChunk;
      } else {
        // buffer exhausted: neutral records (slot 0, length 0) over the part
        // of this chunk inside the buffer; direct adds from now on
        for (uint64_t q = base + (uint64_t)lane; q < Q->jrec_cap && q < base + kRecChunk; q += 64)
          __builtin_nontemporal_store(0ull, &Q->jrec[q]);
        rfull = true;
      }
    }
    if (rfull) {
      for (uint32_t q = done + (uint32_t)lane; q < n; q += 64) {
        const unsigned long long r = rec[q];
        atomicAdd(&Q->jq[r >> kRecValBits], r & ((1ull << kRecValBits) - 1ull));
      }
      return;
    }
    const uint32_t take = (uint64_t)(n - done) < rleft ? n - done : (uint32_t)rleft;
    // records are written once and read back by the next kernels:
    // non-temporal, so they stream past the L2 lines of the grid and tables
    // that the march gathers from
    for (uint32_t q = (uint32_t)lane; q < take; q += 64)
      __builtin_nontemporal_store(rec[done + q], &Q->jrec[rcur + q]);
    rcur += take;
    rleft -= take;
    done += take;
  }
}

constexpr uint64_t kChunk = 128;   // packet ids claimed per atomic on the shared counter
// Interactions and launches are long, divergent branches; run for the one or
// two lanes that need them in a given step they would stall the other lanes
// of the wave nearly every step.  A lane that reaches its interaction point
// holds there until at least 1/kHoldFrac of the wave's live lanes hold, and
// dead lanes are relaunched kRefillMin at a time (or when none is alive).
// Histories do not change: random numbers are keyed by packet id and event.
// With the march loop below, refills of 32 lanes beat 16 by 3.5 % on the
// 256^3 disk (24: 2.5 %, 40: as 32); holding for 1/3 or 1/6 instead of 1/4
// of the live lanes does not pay.
constexpr int kHoldFrac = 4;
constexpr int kRefillMin = 32;

// Packet state: current leaf (integer lower corner lo* in finest units, level
// lev) and the position u* relative to that corner in base-cube units, so that
// rounding scales with the cell, not with the distance from the grid origin;
// crossing into a neighbour re-bases u by an exact integer offset.
// With the deferred path tally (DEFER) the record logic needs more registers:
// five waves per SIMD (a few loop-invariant words spilled, read back only off
// the march) beat six or seven with more spills.
template <typename R, bool TRACE, bool IMG, bool DEFER>
__global__ void __launch_bounds__(256, DEFER ? 5 : 7) k_transport(const TP<R> P) {
  extern __shared__ double smem[];
  __shared__ unsigned int s_cnt[12];
  __shared__ unsigned long long s_stage[DEFER ? 4 * kStage : 1];
  double* s_alb = smem;
  double* s_src = s_alb + P.nl;
  R* s_kext = reinterpret_cast<R*>(s_src + P.nl);
  if (threadIdx.x < 12) s_cnt[threadIdx.x] = 0u;
  for (int j = threadIdx.x; j < P.nl; j += blockDim.x) {
    s_alb[j] = P.albedo[j];
    s_src[j] = P.src_cdf[j];
    s_kext[j] = sizeof(R) == 8 ? (R)P.kext64[j] : (R)P.kext32[j];
  }
  __syncthreads();

  const int lane = __lane_id();
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  const int L = P.L;
  const R inv_nf = P.inv_nf;
  const uint32_t key0 = (uint32_t)P.seed, key1 = (uint32_t)(P.seed >> 32);
  const bool tally_j = (P.flags & MCRT_FLAG_TALLY_J) && P.jq != nullptr;

  bool alive = false, exhausted = false;
  // wave-uniform range [q_next, q_end) of packet ids this wave has claimed:
  // ids are claimed kChunk at a time so the shared counter sees one atomic per
  // kChunk packets instead of one per wave and iteration
  uint64_t q_next = 0, q_end = 0;
  uint64_t pid = 0, kidx = 0;
  uint32_t events = 0;
  R u0 = 0, u1 = 0, u2 = 0, d0 = 0, d1 = 0, d2 = 1, tau = 0, dens = 0;
  // FP32 path: 1/d per axis; -inf for an axis the direction does not move
  // along (1/d not finite), which puts that axis's exit at +inf (or NaN, on
  // its low face, which the minimum below ignores)
  R r0 = 0, r1 = 0, r2 = 1;
  auto set_recip = [&]() {
    if (sizeof(R) == 4) {
      auto one = [](R d) {
        const R q = R(1) / d;
        return __builtin_isfinite(q) ? q : -(R)INFINITY;
      };
      r0 = one(d0);
      r1 = one(d1);
      r2 = one(d2);
    }
  };
  int j = 0, cell = 0, lev = 0, lo0 = 0, lo1 = 0, lo2 = 0;
  // frequent counters in registers, rare ones in LDS
  uint32_t c_cross = 0, c_jseg = 0, c_zero = 0;
  auto bump = [&](int k) { atomicAdd(&s_cnt[k], 1u); };
  // deferred path tally: the wave's current chunk of the record buffer
  // [rcur, rcur + rleft) (wave-uniform); once the buffer is exhausted (rfull)
  // the wave adds to the tally directly
  bool rfull = false;
  unsigned long long* s_rec = s_stage + (threadIdx.x >> 6) * kStage;   // this wave's staging buffer
  uint32_t s_fill = 0u;                                                // records in it (wave-uniform)
  bool hold = false;          // at an interaction point, waiting for the wave's batch
  uint64_t rcur = 0, rleft = 0;
  auto gx = [&](int lo, R u) { return (double)lo * (double)inv_nf + (double)u; };

  for (;;) {
    if (DEFER && s_fill + 64u > kStage) {
      // every lane is here (loop head): the wave's staged records go to the
      // record buffer in bulk when the staging area could not take another
      // full wave of them
      flush_records<R>(s_rec, s_fill, rcur, rleft, rfull);
      s_fill = 0u;
    }
    if (!exhausted || q_next < q_end) {
      const unsigned long long dead = __ballot(!alive);
      if (dead && (__popcll(dead) >= kRefillMin || !__any(alive))) {
        const ArgPtr<R> Q = cold_args<R>();
        const int nd = __popcll(dead);
        if (q_next >= q_end && !exhausted) {
          const int leader = __ffsll((long long)dead) - 1;
          unsigned long long base = 0;
          if (lane == leader) base = atomicAdd(Q->work, (unsigned long long)kChunk);
          base = __shfl(base, leader);
          q_next = base;
          q_end = base + kChunk < Q->n ? base + kChunk : Q->n;
          if (base + kChunk >= Q->n) exhausted = true;
        }
        const uint64_t avail = q_end > q_next ? q_end - q_next : 0;
        const uint64_t rank = (uint64_t)__popcll(dead & lt_mask);
        if (!alive && rank < avail) {
          const uint64_t k = q_next + rank;
          {
            // launch (event slot 0): bin from the source CDF, direction, optical depth
            if (TRACE) kidx = k;
            pid = Q->first_id + k;
            events = 0;
            uint32_t w[4];
            philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), 0u, 0u, key0, key1, w);
            j = cdf_search(s_src, Q->nl, u24(w[0]));
            if (Q->beam_on) { d0 = Q->bx; d1 = Q->by; d2 = Q->bz; }
            else {
              const R mu = (R)(2.0 * u24(w[1]) - 1.0);
              const R st = rsqrt0(R(1) - mu * mu);
              R sp, cp;
              sincos_rev(u24(w[2]), &sp, &cp);
              d0 = st * cp; d1 = st * sp; d2 = mu;
            }
            tau = -rlog((R)u24(w[3]));
            set_recip();
            const double nf = (double)(1 << L);
            cell = locate(P, (int)floor(Q->x0 * nf), (int)floor(Q->y0 * nf), (int)floor(Q->z0 * nf),
                          lev, lo0, lo1, lo2, dens);
            const double ifn = (double)inv_nf;
            u0 = (R)(Q->x0 - (double)lo0 * ifn);
            u1 = (R)(Q->y0 - (double)lo1 * ifn);
            u2 = (R)(Q->z0 - (double)lo2 * ifn);
            bump(0);
            if (IMG && Q->peel_q && cell >= 0 && !Q->beam_on)
              peel_push(Q->x0, Q->y0, Q->z0, cell, j, 0, d0, d1, d2);
            if (TRACE) record(P, kidx, 0, cell, j, Q->x0, Q->y0, Q->z0, d0, d1, d2, tau);
            if (cell < 0) {
              bump(1);
              escape_tally(d0, d1, d2, j);
              if (IMG) image_tally(Q->x0, Q->y0, Q->z0, d0, d1, d2, j);
              if (TRACE) record(P, kidx, 4, -1, j, Q->x0, Q->y0, Q->z0, d0, d1, d2, tau);
            } else {
              alive = true;
            }
          }
        }
        q_next += (uint64_t)nd < avail ? (uint64_t)nd : avail;
      }
    }
    if (!__any(alive)) {
      if (exhausted && q_next >= q_end) break;
      continue;
    }
    // ---- the march: each live lane that is not held steps segment by
    // segment until it holds at an interaction point or leaves the grid, and
    // the wave stops marching once enough lanes hold for a batch, enough lanes
    // are dead for a refill, or the staging area could not take another
    // wave's records.  A lane's state is updated in place here (a lane leaves
    // the loop instead of skipping a block in it).
    {
      int n_alive = __popcll(__ballot(alive));
      int n_hold = __popcll(__ballot(hold));
      const bool can_refill = !exhausted || q_next < q_end;
      uint32_t fill = s_fill;
      if (alive && !hold) {
        for (;;) {
          unsigned long long prec = 0;
          bool hrec = false;
          // ---- one segment: exit distance from the current leaf (lowest axis wins ties)
          const int span = 1 << (L - lev);
          const R side = (R)span * inv_nf;
          R tex = (R)INFINITY;
          int ax = -1;
          if (sizeof(R) == 4) {
            // FP32: the distance to the face the direction points to, per axis,
            // by the direction's reciprocals (one rounding more than a division,
            // well inside FP32 geometry tolerance), negative distances clamped to
            // 0; an axis not moved along gives +inf or NaN, and the minimum skips
            // a NaN.  The lowest axis wins ties.  No branches.
            auto dist = [](R w, R r) { const R x = w * r; return !(x <= R(0)) ? x : R(0); };
            const R t0 = dist(d0 > R(0) ? side - u0 : -u0, r0);
            const R t1 = dist(d1 > R(0) ? side - u1 : -u1, r1);
            const R t2 = dist(d2 > R(0) ? side - u2 : -u2, r2);
            tex = fmin(t0, fmin(t1, t2));
            ax = t0 == tex ? 0 : (t1 == tex ? 1 : 2);
          } else {
            // FP64: divide, as the definition does
            R t;
            if (d0 != R(0)) {
              t = (d0 > R(0) ? side - u0 : -u0) / d0;
              t = t < R(0) ? R(0) : t;
              if (t < tex) { tex = t; ax = 0; }
            }
            if (d1 != R(0)) {
              t = (d1 > R(0) ? side - u1 : -u1) / d1;
              t = t < R(0) ? R(0) : t;
              if (t < tex) { tex = t; ax = 1; }
            }
            if (d2 != R(0)) {
              t = (d2 > R(0) ? side - u2 : -u2) / d2;
              t = t < R(0) ? R(0) : t;
              if (t < tex) { tex = t; ax = 2; }
            }
          }
          const bool dusty = dens > R(0);
          const R alpha = sizeof(R) == 8 ? (R)((double)dens * (double)s_kext[j] * P.h)
                                         : (R)(dens * s_kext[j]);

          if (alpha > R(0) && tau < alpha * tex) {
            // ---- interaction inside this cell
            const R s = tau / alpha;
            u0 += s * d0; u1 += s * d1; u2 += s * d2;
            if (tally_j && dusty) {
              // lengths are below 2^24 units of the finest cell / 2^16
              const unsigned long long q = (unsigned long long)(uint32_t)rrint(s * P.qscale);
              if (DEFER) {
                prec = ((unsigned long long)((uint64_t)(uint32_t)j * (uint64_t)P.n_cells + (uint32_t)cell)
                        << kRecValBits) | q;
                hrec = true;
              } else {
                atomicAdd(&P.jq[(int64_t)j * P.n_cells + cell], q);
              }
              c_jseg++;
            }
            hold = true;
          } else {
            // ---- cross the face into the neighbour
            if (alpha > R(0)) tau -= alpha * tex;
            if (tally_j && dusty) {
              // lengths are below 2^24 units of the finest cell / 2^16
              const unsigned long long q = (unsigned long long)(uint32_t)rrint(tex * P.qscale);
              if (DEFER) {
                prec = ((unsigned long long)((uint64_t)(uint32_t)j * (uint64_t)P.n_cells + (uint32_t)cell)
                        << kRecValBits) | q;
                hrec = true;
              } else {
                atomicAdd(&P.jq[(int64_t)j * P.n_cells + cell], q);
              }
              c_jseg++;
            }
            c_cross++;
            if (tex == R(0)) c_zero++;
            u0 += tex * d0; u1 += tex * d1; u2 += tex * d2;
            const R nf = (R)(1 << L);
            int G0, G1, G2;
            {
              const int f0 = (int)rfloor(u0 * nf), f1 = (int)rfloor(u1 * nf), f2 = (int)rfloor(u2 * nf);
              G0 = lo0 + (f0 < 0 ? 0 : (f0 > span - 1 ? span - 1 : f0));
              G1 = lo1 + (f1 < 0 ? 0 : (f1 > span - 1 ? span - 1 : f1));
              G2 = lo2 + (f2 < 0 ? 0 : (f2 > span - 1 ? span - 1 : f2));
            }
            if (ax == 0) {
              u0 = d0 > R(0) ? side : R(0);
              G0 = d0 > R(0) ? lo0 + span : lo0 - 1;
            } else if (ax == 1) {
              u1 = d1 > R(0) ? side : R(0);
              G1 = d1 > R(0) ? lo1 + span : lo1 - 1;
            } else {
              u2 = d2 > R(0) ? side : R(0);
              G2 = d2 > R(0) ? lo2 + span : lo2 - 1;
            }
            const int o0 = lo0, o1 = lo1, o2 = lo2;
            cell = locate(P, G0, G1, G2, lev, lo0, lo1, lo2, dens);
            if (cell < 0) {
              bump(1);
              alive = false;
              escape_tally(d0, d1, d2, j);
              if (IMG) image_tally(gx(o0, u0), gx(o1, u1), gx(o2, u2), d0, d1, d2, j);
              if (TRACE) record(P, kidx, 4, -1, j, gx(o0, u0), gx(o1, u1), gx(o2, u2), d0, d1, d2, tau);
            } else {
              // re-base the local position on the new leaf (exact integer offsets)
              u0 += (R)(o0 - lo0) * inv_nf;
              u1 += (R)(o1 - lo1) * inv_nf;
              u2 += (R)(o2 - lo2) * inv_nf;
              if (TRACE) record(P, kidx, 1, cell, j, gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), d0, d1, d2, tau);
            }
          }

          if (DEFER) {
            // the marching lanes' records go to the wave's LDS staging area,
            // in lane order.  A record store to global memory per step would
            // be waited for by the step's next wait on memory (vector memory
            // operations are counted in issue order): a write round trip per
            // step, which an LDS store is not.
            const unsigned long long rm = __ballot(hrec);
            if (hrec) s_rec[fill + (uint32_t)__popcll(rm & lt_mask)] = prec;
            fill += (uint32_t)__popcll(rm);
          }
          n_hold += __popcll(__ballot(hold));
          n_alive -= __popcll(__ballot(!alive));
          if (!alive || hold) break;
          if (n_hold * kHoldFrac >= n_alive || (can_refill && 64 - n_alive >= kRefillMin) ||
              (DEFER && fill + 64u > kStage))
            break;
        }
      }
      // lanes left the march at different steps: the last count is the largest
      if (DEFER) s_fill = wave_max_u32(fill);
    }

    // ---- the wave's held interactions, once enough lanes hold
    {
      const unsigned long long hm = __ballot(hold);
      if (hm && __popcll(hm) * kHoldFrac >= __popcll(__ballot(alive))) {
        if (hold) {
          const ArgPtr<R> Q = cold_args<R>();
          hold = false;
          events += 1;
          if ((uint64_t)events > Q->max_events) {
            bump(2);
            alive = false;
            if (TRACE) record(P, kidx, 5, cell, j, gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), d0, d1, d2, tau);
            continue;
          }
          uint32_t w[4];
          philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), events, 0u, key0, key1, w);
          R sp, cp;
          sincos_rev(u24(w[2]), &sp, &cp);
          if (u24(w[0]) <= s_alb[j]) {
            // scattering: new direction from the phase function
            if (IMG && Q->peel_q) peel_push(gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), cell, j, 1, d0, d1, d2);
            const R mu = (R)hg_mu(Q->gpar[j], u24(w[1]));
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
            bump(4);
            set_recip();
            tau = -rlog((R)u24(w[3]));
            if (TRACE) record(P, kidx, 2, cell, j, gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), d0, d1, d2, tau);
          } else {
            // absorption: species, tally, new frequency, isotropic re-emission
            uint32_t v[4];
            philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), events, 1u, key0, key1, v);
            const int sp_i = cdf_search(Q->sp_cdf + (int64_t)j * Q->S, Q->S, u24(w[1]));
            unsigned long long before = atomicAdd(&Q->nabs[(int64_t)cell * Q->S + sp_i], 1ull);
            bump(5);
            if (Q->flags & MCRT_FLAG_FROZEN_T) before = Q->frozen[(int64_t)cell * Q->S + sp_i];
            if (Q->flags & MCRT_FLAG_KILL_ON_ABSORB) {
              bump(3);
              alive = false;
              if (TRACE) record(P, kidx, 3, cell, j, gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), d0, d1, d2, tau);
              continue;
            }
            if (Q->kind[sp_i] == 0) {
              // Bracket of the absorbed energy; with the exact Bjorkman-Wood form
              // a point uniform between the energies before and after this
              // absorption, which picks the rows spanning T_before..T_after in
              // proportion to the energy each covers.
              const double vol = ldexp(Q->h3, -3 * lev);
              double nb = (double)before;
              if (Q->flags & MCRT_FLAG_EXACT_BW) nb += u24(v[2]);
              const double pw = nb * Q->eps / (Q->rho[cell] * vol);
              const double* E = Q->E + (int64_t)sp_i * Q->K;
              int kb;
              if (pw < E[0]) {
                kb = 0;
                bump(7);
              } else {
                int a = 0, b = Q->K - 1;
                if (E[Q->K - 1] <= pw) a = Q->K - 1;
                else
                  while (b - a > 1) {
                    const int m = (a + b) >> 1;
                    if (E[m] <= pw) a = m; else b = m;
                  }
                kb = a;
                if (kb > Q->K - 2) { kb = Q->K - 2; bump(8); }
              }
              j = cdf_search(Q->Rrows + ((int64_t)sp_i * (Q->K - 1) + kb) * Q->nl, Q->nl, u24(v[0]));
            } else {
              const double* row = Q->pah_rows + ((int64_t)Q->pah_slot[sp_i] * P.n_cells + cell) * Q->nl;
              j = cdf_search(row, Q->nl, u24(v[0]));
              bump(9);
            }
            const R mu = (R)(2.0 * u24(v[1]) - 1.0);
            const R st = rsqrt0(R(1) - mu * mu);
            d0 = st * cp; d1 = st * sp; d2 = mu;
            set_recip();
            tau = -rlog((R)u24(w[3]));
            if (IMG && Q->peel_q) peel_push(gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), cell, j, 0, d0, d1, d2);
            if (TRACE) record(P, kidx, 3, cell, j, gx(lo0, u0), gx(lo1, u1), gx(lo2, u2), d0, d1, d2, tau);
          }
        }
      }
    }
  }

  if (DEFER) {
    if (s_fill) flush_records<R>(s_rec, s_fill, rcur, rleft, rfull);
    // the unused tail of the wave's last chunk holds neutral records
    if (!rfull)
      for (uint64_t q = (uint64_t)lane; q < rleft; q += 64) __builtin_nontemporal_store(0ull, &P.jrec[rcur + q]);
  }

  // ---- counters: registers reduced per wave, LDS per block
  {
    const unsigned long long s6 = wave_sum((unsigned long long)c_cross);
    const unsigned long long s10 = wave_sum((unsigned long long)c_zero);
    const unsigned long long s11 = wave_sum((unsigned long long)c_jseg);
    if (lane == 0) {
      if (s6) atomicAdd(&P.counters[6], s6);
      if (s10) atomicAdd(&P.counters[10], s10);
      if (s11) atomicAdd(&P.counters[11], s11);
    }
  }
  __syncthreads();
  if (threadIdx.x < 12 && s_cnt[threadIdx.x])
    atomicAdd(&P.counters[threadIdx.x], (unsigned long long)s_cnt[threadIdx.x]);
}

// Next-event march: one lane per (record, observer).  Optical depth from the
// record's position along the line of sight to the edge of the grid, cell by
// cell with the transport's face rules, then the weight (phase function for a
// scattering, times exp(-tau)) added in fixed point at the record's pixel.
// Every lane ends: each step moves the finest-level index along the exit axis
// by at least one in the direction of travel, and a step cap bounds the march.
template <typename R>
__global__ void __launch_bounds__(256) k_peel(const TP<R> P) {
  const unsigned long long cnt = *P.peel_count;
  const uint64_t n_rec = cnt < P.peel_cap ? cnt : P.peel_cap;
  const ImgP& I = P.img;
  const int n_obs = I.n_obs, L = P.L;
  const uint64_t total = n_rec * (uint64_t)n_obs;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const R inv_nf = P.inv_nf;
  const R nf = (R)(1 << L);
  const int max_steps = 4 * (P.nb << L) + 64;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const uint64_t k = i / (uint64_t)n_obs;
    const int o = (int)(i - k * (uint64_t)n_obs);
    const PeelRec r = reinterpret_cast<const PeelRec*>(P.peel_q)[k];
    const int j = r.j;
    int l = -1;
    for (int q = 0; q < I.n_l; ++q)
      if (I.lsel[q] == j) l = q;
    const bool sed = P.peel_sed != nullptr;
    if (l < 0 && !sed) continue;
    const double X0 = I.off[0] + r.x[0] * I.h, X1 = I.off[1] + r.x[1] * I.h, X2 = I.off[2] + r.x[2] * I.h;
    const double a = X0 * I.e1[o][0] + X1 * I.e1[o][1] + X2 * I.e1[o][2];
    const double b = X0 * I.e2[o][0] + X1 * I.e2[o][1] + X2 * I.e2[o][2];
    const double fx = floor((a + I.w) / (2.0 * I.w) * I.npix), fy = floor((b + I.w) / (2.0 * I.w) * I.npix);
    const bool in_img = l >= 0 && !(fx < 0.0 || fy < 0.0 || fx >= I.npix || fy >= I.npix);
    if (!in_img && !sed) continue;
    double ph = 1.0;
    if (r.type == 1) {
      const double g = P.gpar[j];
      if (fabs(g) >= 1e-5) {
        const double mu = r.din[0] * I.n[o][0] + r.din[1] * I.n[o][1] + r.din[2] * I.n[o][2];
        const double den = 1.0 + g * g - 2.0 * g * mu;
        ph = (1.0 - g * g) / (den * sqrt(den));
      }
    }
    const R n0 = (R)I.n[o][0], n1 = (R)I.n[o][1], n2 = (R)I.n[o][2];
    const R kx = sizeof(R) == 8 ? (R)P.kext64[j] : (R)P.kext32[j];
    int cell = r.cell, lev = P.level[cell];
    const int4 lo4 = P.leaf_lo[cell];
    int lo0 = lo4.x, lo1 = lo4.y, lo2 = lo4.z;
    R dens = sizeof(R) == 8 ? (R)P.rho[cell] : (R)P.rho_h32[cell];
    R u0 = (R)(r.x[0] - (double)lo0 * (double)inv_nf);
    R u1 = (R)(r.x[1] - (double)lo1 * (double)inv_nf);
    R u2 = (R)(r.x[2] - (double)lo2 * (double)inv_nf);
    R tau = 0;
    for (int step = 0; step < max_steps; ++step) {
      const int span = 1 << (L - lev);
      const R side = (R)span * inv_nf;
      R tex = (R)INFINITY;
      int ax = 0;
      R t;
      if (n0 != R(0)) {
        t = (n0 > R(0) ? side - u0 : -u0) / n0;
        t = t < R(0) ? R(0) : t;
        if (t < tex) { tex = t; ax = 0; }
      }
      if (n1 != R(0)) {
        t = (n1 > R(0) ? side - u1 : -u1) / n1;
        t = t < R(0) ? R(0) : t;
        if (t < tex) { tex = t; ax = 1; }
      }
      if (n2 != R(0)) {
        t = (n2 > R(0) ? side - u2 : -u2) / n2;
        t = t < R(0) ? R(0) : t;
        if (t < tex) { tex = t; ax = 2; }
      }
      const R alpha = sizeof(R) == 8 ? (R)((double)dens * (double)kx * P.h) : dens * kx;
      tau += alpha * tex;
      u0 += tex * n0; u1 += tex * n1; u2 += tex * n2;
      int G0, G1, G2;
      {
        const int f0 = (int)rfloor(u0 * nf), f1 = (int)rfloor(u1 * nf), f2 = (int)rfloor(u2 * nf);
        G0 = lo0 + (f0 < 0 ? 0 : (f0 > span - 1 ? span - 1 : f0));
        G1 = lo1 + (f1 < 0 ? 0 : (f1 > span - 1 ? span - 1 : f1));
        G2 = lo2 + (f2 < 0 ? 0 : (f2 > span - 1 ? span - 1 : f2));
      }
      if (ax == 0) {
        u0 = n0 > R(0) ? side : R(0);
        G0 = n0 > R(0) ? lo0 + span : lo0 - 1;
      } else if (ax == 1) {
        u1 = n1 > R(0) ? side : R(0);
        G1 = n1 > R(0) ? lo1 + span : lo1 - 1;
      } else {
        u2 = n2 > R(0) ? side : R(0);
        G2 = n2 > R(0) ? lo2 + span : lo2 - 1;
      }
      const int o0 = lo0, o1 = lo1, o2 = lo2;
      cell = locate(P, G0, G1, G2, lev, lo0, lo1, lo2, dens);
      if (cell < 0) break;
      u0 += (R)(o0 - lo0) * inv_nf;
      u1 += (R)(o1 - lo1) * inv_nf;
      u2 += (R)(o2 - lo2) * inv_nf;
    }
    const double wgt = ph * exp(-(double)tau);
    const unsigned long long q = (unsigned long long)rint(wgt * MCRT_PEEL_UNIT);
    if (in_img) atomicAdd(&P.peel[(((int64_t)o * I.n_l + l) * I.npix + (int64_t)fy) * I.npix + (int64_t)fx], q);
    // the observer's next-event SED: every bin, wherever the event projects
    if (sed) atomicAdd(&P.peel_sed[(int64_t)o * P.nl + j], q);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (cnt) atomicAdd(&P.counters[MCRT_CNT_PEEL], cnt);
    if (cnt > P.peel_cap) atomicAdd(&P.counters[MCRT_CNT_PEEL_DROPPED], cnt - P.peel_cap);
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
  P.h3 = d.base_size * d.base_size * d.base_size;
  P.eps = c->src.lum / (double)o.n_total;
  P.x0 = (c->src.pos[0] - d.box_min[0]) / d.base_size;
  P.y0 = (c->src.pos[1] - d.box_min[1]) / d.base_size;
  P.z0 = (c->src.pos[2] - d.box_min[2]) / d.base_size;
  P.bx = (R)c->src.beam[0]; P.by = (R)c->src.beam[1]; P.bz = (R)c->src.beam[2];
  P.first_id = first_id; P.n = n; P.seed = o.seed; P.max_events = o.max_events;
  P.base_map = d.base_map; P.nodes = d.nodes; P.rho = d.rho;
  P.binfo = reinterpret_cast<const int2*>(T + L.binfo);
  P.rho_h32 = reinterpret_cast<const float*>(T + L.rho_h32);
  P.kext64 = reinterpret_cast<const double*>(T + L.kext);
  P.kext32 = reinterpret_cast<const float*>(T + L.kext32);
  P.albedo = reinterpret_cast<const double*>(T + L.albedo);
  P.gpar = reinterpret_cast<const double*>(T + L.gpar);
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
  P.img = c->img;
  P.img.image = reinterpret_cast<unsigned long long*>(t.image);
  const bool img = c->img.n_obs > 0;
  const bool peel = img && (o.flags & MCRT_FLAG_PEEL);
  if (peel) {
    P.peel_q = static_cast<unsigned char*>(o.peel_queue);
    P.peel_cap = o.peel_capacity;
    P.peel_count = &scr->peel_count;
    P.level = reinterpret_cast<const int8_t*>(T + L.level);
    P.leaf_lo = reinterpret_cast<const int4*>(T + L.leaf_lo);
    P.peel = reinterpret_cast<unsigned long long*>(t.peel);
    P.peel_sed = (o.flags & MCRT_FLAG_PEEL_SED) ? reinterpret_cast<unsigned long long*>(t.peel_sed) : nullptr;
    k_zero_u64<<<1, 64, 0, s>>>(&scr->peel_count, 1);
  }
  k_zero_u64<<<1, 64, 0, s>>>(&scr->work_counter, 1);
  const uint64_t want = (n + 255) / 256;
  const size_t lds = (size_t)d.n_lambda * (2 * sizeof(double) + sizeof(R));
  // persistent grid: as many blocks as can be resident at once
  const bool defer = o.jrec_ws != nullptr && (o.flags & MCRT_FLAG_TALLY_J) && t.jq != nullptr;
  if (defer) {
    const JrecLayout J = jrec_layout((uint64_t)d.n_lambda * (uint64_t)d.n_cells, o.jrec_capacity);
    unsigned char* ws = static_cast<unsigned char*>(o.jrec_ws);
    P.jrec = reinterpret_cast<unsigned long long*>(ws + J.recA);
    P.jrec_cap = J.capacity;
    P.jrec_count = reinterpret_cast<unsigned long long*>(ws + J.hdr);
    k_zero_u64<<<1, 64, 0, s>>>(P.jrec_count, 8);
  }
  auto kern = o.trace ? (img ? k_transport<R, true, true, false> : k_transport<R, true, false, false>)
              : defer ? (img ? k_transport<R, false, true, true> : k_transport<R, false, false, true>)
                      : (img ? k_transport<R, false, true, false> : k_transport<R, false, false, false>);
  int per_cu = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds);
  if (per_cu < 1) per_cu = 1;
  uint64_t blocks = o.grid_blocks > 0 ? (uint64_t)o.grid_blocks : (uint64_t)c->n_cu * per_cu;
  if (blocks > want) blocks = want;
  if (blocks < 1) blocks = 1;
  if (o.kernel_begin) {
    const hipError_t e = hipEventRecord(o.kernel_begin, s);
    if (e != hipSuccess) return e;
  }
  kern<<<(unsigned)blocks, 256, lds, s>>>(P);
  if (o.kernel_end) {
    const hipError_t e = hipEventRecord(o.kernel_end, s);
    if (e != hipSuccess) return e;
  }
  if (peel) k_peel<R><<<(unsigned)(c->n_cu * 4), 256, 0, s>>>(P);
  if (defer) {
    const hipError_t e = launch_jrec_accumulate(c, o, first_id, n, t.jq, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_transport(mcrt_ctx* c, uint64_t first_id, uint64_t n, const mcrt_run_opts& o,
                            const mcrt_tallies& t, hipStream_t s) {
  if (c->d.precision == MCRT_F64) return launch_t<double>(c, first_id, n, o, t, s);
  return launch_t<float>(c, first_id, n, o, t, s);
}

}  // namespace mcrt
