// Exact steady-state temperature distribution P(T) of transiently heated PAHs
// and their band/continuum emission, per cell, in FP64 (paper Sec. 1, Sec. 4,
// Fig. 3: P(T) depends on the strength and the hardness of the field).
//
// Heating: the N_j = 4 pi C_j J_j dnu_j / (h nu_j) photons per second of
// wavelength bin j move a molecule from U_i to x = U_i + E_j (E_j = h nu_j),
// shared between the two bin centres around x so that the mean gain is E_j.
// The steady state needs only the cumulative upward rates
//   B_{f,i} = sum_{k>=f} A_{k,i}
//           = C[m(f,i)] + sum_{m(f,i) <= j < m(f-1,i)} N_j (U_i + E_j - U_{f-1}) / dU_f,
// with m(f,i) = #{j : U_f <= U_i + E_j} (photon energy falls with j, so these
// j lead) and C[m] = sum_{j<m} N_j; for i = f-1 the second sum runs over all
// j >= m(f,i) and equals H[m] / dU_f, H[m] = sum_{j>=m} N_j E_j.  Every B is
// thus a sum of positive terms read from two per-cell prefix arrays and a
// cell-independent index table: no running subtraction, no per-cell matrix.
//
// Recurrence P_f dU_f^-1 P_em(T_f) = sum_{i<f} P_i B_{f,i}, P_0 = 1, in blocks
// of kBk values of f: the contribution of earlier blocks (X_f) is a
// matrix-vector product over all threads, the in-block part runs on one wave
// per cell with the block's B entries staged in LDS.  Four cells per
// 256-thread workgroup share every table load.
#include <cmath>
#include <cstdio>
#include <new>
#include <string>

#include "mcrt_internal.h"
#include "pah.h"
#include "pah_internal.h"

using namespace mcrt;

namespace {

constexpr int kBk = 32;
constexpr int kThreads = 256;
constexpr int kNC = 4;             // cells per workgroup

constexpr int kBpBlocks = 256;        // partial sums of the band-power reduction

struct PahLayout {
  uint64_t nu, dnu, ed, E, fac, invdu, mtab, adown, em, bandw, bp_part, total;
};

PahLayout pah_layout(const pah_desc& d) {
  PahLayout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t b) {
    const uint64_t o = off;
    off += (b + 255) & ~uint64_t(255);
    return o;
  };
  const uint64_t M = d.M, nl = d.n_lambda, no = (uint64_t)d.n_bands + nl;
  L.nu = take(8 * nl);
  L.dnu = take(8 * nl);
  L.ed = take(8 * (nl + 1));
  L.E = take(8 * nl);
  L.fac = take(8 * nl);
  L.invdu = take(8 * M);
  L.mtab = take(4 * M * M);
  L.adown = take(8 * M);
  L.em = take(8 * M * no);
  L.bandw = take(8 * (uint64_t)(d.n_bands > 0 ? d.n_bands : 1) * nl);
  L.bp_part = take(8 * (uint64_t)kBpBlocks * 64);
  L.total = off;
  return L;
}

// wavelength bins: centres, widths, edges (micron), photon energies and the
// factor 4 pi dnu / (h nu) turning C J into photons per second; 1 / dU_f
__global__ void k_pah_bins(int nl, int M, const double* __restrict__ lam, const double* __restrict__ U,
                           double* nu, double* dnu, double* ed, double* E, double* fac, double* invdu) {
  for (int j = threadIdx.x; j <= nl; j += blockDim.x) {
    double e;
    if (j == 0) e = lam[0] * lam[0] / sqrt(lam[0] * lam[1]);
    else if (j == nl) e = lam[nl - 1] * lam[nl - 1] / sqrt(lam[nl - 2] * lam[nl - 1]);
    else e = sqrt(lam[j - 1] * lam[j]);
    ed[j] = e;
  }
  for (int f = threadIdx.x; f < M; f += blockDim.x) invdu[f] = f > 0 ? 1.0 / (U[f] - U[f - 1]) : 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    nu[j] = kC / (lam[j] * 1e-4);
    dnu[j] = kC / (ed[j] * 1e-4) - kC / (ed[j + 1] * 1e-4);
    E[j] = kH * nu[j];
    fac[j] = 4.0 * kPi * dnu[j] / E[j];
  }
}

// m(f,i) = number of wavelength bins whose photons lift state i to U_f or
// beyond (a leading run of j: the photon energy falls with j)
__device__ int count_reaching(int nl, const double* __restrict__ E, double Ui, double Uf) {
  int lo = 0, hi = nl;                   // first j with U_i + E_j < U_f
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Uf <= Ui + E[mid]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// both counts a pair (f, i), f > i, needs, in one word:
// m(f,i) | m(f-1,i) << 16 (the high half is 0 for i = f-1)
__global__ void k_pah_m(int M, int nl, const double* __restrict__ U, const double* __restrict__ E,
                        uint32_t* __restrict__ mtab) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * M) return;
  const int f = (int)(q / M), i = (int)(q % M);
  uint32_t v = 0;
  if (i < f) {
    v = (uint32_t)count_reaching(nl, E, U[i], U[f]);
    if (i < f - 1) v |= (uint32_t)count_reaching(nl, E, U[i], U[f - 1]) << 16;
  }
  mtab[q] = v;
}

// cooling rates and emission table
__global__ void k_pah_em(int M, int nl, int nbd, const double* __restrict__ T,
                         const double* __restrict__ U, const double* __restrict__ nu,
                         const double* __restrict__ dnu, const double* __restrict__ cabs,
                         const double* __restrict__ cband, const double* __restrict__ ccont,
                         double* __restrict__ adown, double* __restrict__ em) {
  const int i = blockIdx.x;
  const int no = nbd + nl;
  __shared__ double red[256];
  double pe = 0.0;
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    const double B = planck_nu(nu[j], T[i]);
    pe += cabs[j] * B * dnu[j];
    em[(int64_t)i * no + nbd + j] = 4.0 * kPi * ccont[j] * B * dnu[j];
  }
  red[threadIdx.x] = pe;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) adown[i] = i > 0 ? 4.0 * kPi * red[0] / (U[i] - U[i - 1]) : 0.0;
  for (int b = threadIdx.x; b < nbd; b += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nl; ++j) s += cband[(int64_t)b * nl + j] * planck_nu(nu[j], T[i]) * dnu[j];
    em[(int64_t)i * no + b] = 4.0 * kPi * s;
  }
}

// band profile on the grid: Cband_b(j) dnu_j normalised over j
__global__ void k_pah_bandw(int nl, const double* __restrict__ cband, const double* __restrict__ dnu,
                            double* __restrict__ w) {
  const int b = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < nl; j += blockDim.x) s += cband[(int64_t)b * nl + j] * dnu[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double tot = red[0];
  for (int j = threadIdx.x; j < nl; j += blockDim.x)
    w[(int64_t)b * nl + j] = tot > 0.0 ? cband[(int64_t)b * nl + j] * dnu[j] / tot : 0.0;
}

// re-emission CDF row per cell: continuum power per bin plus band powers
// spread by their profiles, running sum normalised to end at exactly 1.
// Persistent grid, one wave per cell at a time: the band profiles are staged
// in LDS once per workgroup (when they fit), a cell's band powers are
// wave-uniform scalar loads, chunks of 64 bins are scanned with shuffles, and
// the running sums stay in registers for up to 256 bins (parked in `rows`
// beyond that) until the total is known.
constexpr int kRowLdsMax = 48 * 1024;

template <bool W_IN_LDS>
__global__ void __launch_bounds__(256) k_pah_rows(int nl, int nbd, int64_t n, const double* __restrict__ out,
                                                  const double* __restrict__ wg, double* __restrict__ rows) {
  extern __shared__ double sw[];                      // [nbd][nl] when W_IN_LDS
  if (W_IN_LDS) {
    for (int q = threadIdx.x; q < nbd * nl; q += blockDim.x) sw[q] = wg[q];
    __syncthreads();
  }
  const double* w = W_IN_LDS ? sw : wg;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int no = nbd + nl;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < n; c += (int64_t)gridDim.x * 4) {
    const double* o = out + c * no;
    double* r = rows + c * nl;
    double keep[4];
    double carry = 0.0;
    for (int base = 0, ch = 0; base < nl; base += 64, ++ch) {
      const int j = base + lane;
      double e = 0.0;
      if (j < nl) {
        e = o[nbd + j];
        for (int bd = 0; bd < nbd; ++bd) e += o[bd] * w[bd * nl + j];
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(e, off);
        if (lane >= off) e += y;
      }
      e += carry;
      if (ch < 4) keep[ch & 3] = e;
      else if (j < nl) r[j] = e;
      carry = __shfl(e, 63);
    }
    const double tot = carry;
    for (int base = 0, ch = 0; base < nl; base += 64, ++ch) {
      const int j = base + lane;
      if (j >= nl) break;
      const double e = ch < 4 ? keep[ch & 3] : r[j];
      r[j] = (j == nl - 1 || !(tot > 0.0)) ? 1.0 : e / tot;
    }
  }
}

struct SolveP {
  int M, nl, nbd, nblk, j_f32;
  int64_t n;
  const void* J;
  const double* cabs;
  const double* U;
  const double* E;
  const double* fac;
  const double* invdu;
  const uint32_t* mtab;   // m(f,i) | m(f-1,i) << 16
  const double* adown;
  const double* em;
  double* out;
  double* P_out;
  double* pabs;
  const int64_t* idx;     // cells to solve (null: 0..n-1)
  const int64_t* n_dev;   // device count of idx (null: n)
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// The per-cell LDS arrays interleave the kNC = 4 cells ([index][cell]), so the
// four values at one index are two 16-byte LDS reads.
static_assert(kNC == 4, "the LDS gathers read four cells at a time");
__device__ __forceinline__ void ld4(const double* p, double* v) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void ld4_add(const double* p, double s, double* acc) {
  double v[4];
  ld4(p, v);
#pragma unroll
  for (int w = 0; w < 4; ++w) acc[w] += s * v[w];
}
__device__ __forceinline__ void ld4_mul_add(const double* p, const double* x, double* acc) {
  double v[4];
  ld4(p, v);
#pragma unroll
  for (int w = 0; w < 4; ++w) acc[w] += v[w] * x[w];
}

// the value of v in lane l (l wave-uniform), for every lane
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ double wave_scan_d(double v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(v, off);
    if (lane >= off) v += y;
  }
  return v;
}

// B_{f,i} (f > i) for the kNC cells of the workgroup, from the counts
// m = m(f,i) and m1 = m(f-1,i) (m1 unused when i = f-1)
// (sU, sInv, sE: the enthalpies, 1/dU and photon energies staged in LDS)
__device__ __forceinline__ void cum_rates_at(const SolveP& P, const double* sN, const double* sC,
                                             const double* sH, const double* sU, const double* sInv,
                                             const double* sE, int f, int i, int m, int m1, double* Bv) {
  const int nl = P.nl;
  ld4(sC + m * kNC, Bv);
  const double inv = sInv[f];
  if (i == f - 1) {
    ld4_add(sH + m * kNC, inv, Bv);
  } else if (m1 > m) {
    const double Ui = sU[i], Uf1 = sU[f - 1];
    for (int j = m; j < m1; ++j) {
      const double wt = ((Ui + sE[j]) - Uf1) * inv;
      ld4_add(sN + j * kNC, wt, Bv);
    }
  }
}

__device__ __forceinline__ void cum_rates(const SolveP& P, const double* sN, const double* sC,
                                          const double* sH, const double* sU, const double* sInv,
                                          const double* sE, int f, int i, double* Bv) {
  const int M = P.M;
  const uint32_t v = P.mtab[(int64_t)f * M + i];
  const int m = (int)(v & 0xFFFFu), m1 = (int)(v >> 16);
  cum_rates_at(P, sN, sC, sH, sU, sInv, sE, f, i, m, m1, Bv);
}

// kNC cells per workgroup: every cell-independent table entry is loaded once
// and applied to kNC cells; the in-block recurrence of cell w runs on wave w.
__global__ void __launch_bounds__(kThreads) k_pah_solve(const SolveP P) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  const int M = P.M, nl = P.nl, nbd = P.nbd, nblk = P.nblk;
  const int no = nbd + nl;
  double* sP = sm;                              // [M][kNC]
  double* sN = sP + kNC * M;                    // [nl][kNC]     photons per second
  double* sC = sN + kNC * nl;                   // [nl + 1][kNC] sum_{j<m} N_j
  double* sH = sC + kNC * (nl + 1);             // [nl + 1][kNC] sum_{j>=m} N_j E_j
  double* sBin = sH + kNC * (nl + 1);           // [kNC][kBk * kBk]
  double* sX = sBin + kNC * kBk * kBk;          // [kNC][kBk]
  double* sU = sX + kNC * kBk;                  // [M]  enthalpies      (shared by the cells)
  double* sInv = sU + M;                        // [M]  1 / (U_f - U_{f-1})
  double* sE = sInv + M;                        // [nl] photon energies
  int* sScale = reinterpret_cast<int*>(sE + nl);          // [kNC]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;

  for (int i = t; i < M; i += kThreads) {
    sU[i] = P.U[i];
    sInv[i] = P.invdu[i];
  }
  for (int j = t; j < nl; j += kThreads) sE[j] = P.E[j];
  __syncthreads();

  const int64_t n_cells = P.n_dev ? *P.n_dev : P.n;
  const int64_t n_groups = (n_cells + kNC - 1) / kNC;
  for (int64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    int64_t cell[kNC];
    bool valid[kNC];
#pragma unroll
    for (int w = 0; w < kNC; ++w) {
      const int64_t cl = grp * kNC + w;
      valid[w] = cl < n_cells;
      cell[w] = valid[w] ? (P.idx ? P.idx[cl] : cl) : -1;
    }
    // ---- photon rates of every wavelength bin
    for (int q = t; q < kNC * nl; q += kThreads) {
      const int w = q / nl, j = q % nl;
      double Jj = 0.0;
      if (valid[w])
        Jj = P.j_f32 ? (double)reinterpret_cast<const float*>(P.J)[cell[w] * nl + j]
                     : reinterpret_cast<const double*>(P.J)[cell[w] * nl + j];
      sN[j * kNC + w] = P.cabs[j] * Jj * P.fac[j];
    }
    __syncthreads();
    // ---- prefix sums C (from the most energetic bin) and H (from the least):
    // wave w scans cell w; H[0] is the absorbed power
    if (wave < kNC) {
      const int w = wave;
      double carry = 0.0;
      if (lane == 0) sC[w] = 0.0;
      for (int base = 0; base < nl; base += 64) {
        const int j = base + lane;
        const double v = wave_scan_d(j < nl ? sN[j * kNC + w] : 0.0, lane) + carry;
        if (j < nl) sC[(j + 1) * kNC + w] = v;
        carry = __shfl(v, 63);
      }
      carry = 0.0;
      if (lane == 0) sH[nl * kNC + w] = 0.0;
      for (int base = 0; base < nl; base += 64) {
        const int j = nl - 1 - (base + lane);
        const double v = wave_scan_d(j >= 0 ? sN[j * kNC + w] * sE[j] : 0.0, lane) + carry;
        if (j >= 0) sH[j * kNC + w] = v;
        carry = __shfl(v, 63);
      }
      if (lane == 0 && P.pabs && valid[w]) P.pabs[cell[w]] = sH[w];
      if (lane == 0) { sP[w] = 1.0; sScale[w] = 0; }
    }
    __syncthreads();

    // ---- blocks of f upward
    for (int b = 0; b < nblk; ++b) {
      const int fb = 1 + kBk * b;
      const int eb = fb + kBk < M ? fb + kBk : M;
      const int bk = eb - fb;
      // X_f = sum_{i<fb} P_i B_{f,i}: 32 f-slots x 8 i-groups, all cells per load
      {
        const int kk = t >> 3, g = t & 7;
        double acc[kNC] = {};
        if (kk < bk) {
          const int f = fb + kk;
          const uint32_t* rowf = P.mtab + (int64_t)f * M;
          int i = g;
          // four states per pass with all index loads issued first
          for (; i + 24 < fb; i += 32) {
            int m[4], m1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint32_t v = rowf[i + 8 * u];
              m[u] = (int)(v & 0xFFFFu);
              m1[u] = (int)(v >> 16);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              double Bv[kNC];
              cum_rates_at(P, sN, sC, sH, sU, sInv, sE, f, i + 8 * u, m[u], m1[u], Bv);
              ld4_mul_add(sP + (i + 8 * u) * kNC, Bv, acc);
            }
          }
          for (; i < fb; i += 8) {
            double Bv[kNC];
            const uint32_t v = rowf[i];
            cum_rates_at(P, sN, sC, sH, sU, sInv, sE, f, i, (int)(v & 0xFFFFu), (int)(v >> 16), Bv);
            ld4_mul_add(sP + i * kNC, Bv, acc);
          }
        }
#pragma unroll
        for (int w = 0; w < kNC; ++w) {
          acc[w] += __shfl_xor(acc[w], 1);
          acc[w] += __shfl_xor(acc[w], 2);
          acc[w] += __shfl_xor(acc[w], 4);
          if (g == 0 && kk < kBk) sX[w * kBk + kk] = kk < bk ? acc[w] : 0.0;
        }
      }
      // in-block entries B_{f,i}, fb <= i < f < eb, column-major: [i - fb][f - fb]
      for (int q = t; q < kBk * kBk; q += kThreads) {
        const int col = q / kBk, fl = q % kBk;
        if (col < fl && fl < bk) {
          double Bv[kNC];
          cum_rates(P, sN, sC, sH, sU, sInv, sE, fb + fl, fb + col, Bv);
#pragma unroll
          for (int w = 0; w < kNC; ++w) sBin[w * kBk * kBk + q] = Bv[w];
        }
      }
      __syncthreads();
      // sequential recurrence, right-looking: wave w for cell w; lane l owns
      // row fb+l and its running sum S of P_i B_{fb+l,i} over solved i of the
      // block; each step divides in the owning lane, broadcasts P_f with
      // v_readlane and updates the later rows with one FMA
      if (wave < kNC) {
        const int w = wave;
        const double* binT = sBin + w * kBk * kBk;
        const double rAl = lane < bk ? 1.0 / P.adown[fb + lane] : 0.0;
        const double Xl = lane < bk ? sX[w * kBk + lane] : 0.0;
        double S = 0.0, myP = 0.0;
        int nsc = 0;                       // rescales by 2^-664 inside this block
        for (int fl = 0; fl < bk; ++fl) {
          const double cand = ((nsc ? ldexp(Xl, -664 * nsc) : Xl) + S) * rAl;
          double Pf = readlane_d(cand, fl);
          if (lane == fl) myP = Pf;
          if (Pf > 1e200) {                 // keep the unnormalised P finite
            ++nsc;
            if (lane <= fl) myP = ldexp(myP, -664);
            S = ldexp(S, -664);
            Pf = ldexp(Pf, -664);
          }
          if (lane > fl && lane < bk) S += Pf * binT[fl * kBk + lane];
        }
        if (lane < bk) sP[(fb + lane) * kNC + w] = myP;
        if (lane == 0) sScale[w] = nsc;
      }
      __syncthreads();
      for (int q = t; q < kNC * fb; q += kThreads) {
        const int w = q / fb, i = q % fb;
        const int nsc = sScale[w];
        if (nsc) sP[i * kNC + w] = ldexp(sP[i * kNC + w], -664 * nsc);
      }
      __syncthreads();
    }

    // ---- normalise (wave w: cell w) and emit
    if (wave < kNC) {
      double tot = 0.0;
      for (int i = lane; i < M; i += 64) tot += sP[i * kNC + wave];
      tot = wave_sum_d(tot);
      for (int i = lane; i < M; i += 64) sP[i * kNC + wave] /= tot;
    }
    __syncthreads();
    if (P.P_out)
      for (int q = t; q < kNC * M; q += kThreads) {
        const int w = q / M, i = q % M;
        if (valid[w]) P.P_out[cell[w] * M + i] = sP[i * kNC + w];
      }
    for (int q = t; q < no; q += kThreads) {
      double acc[kNC] = {};
#pragma unroll 8
      for (int i = 1; i < M; ++i) {
        const double e = P.em[(int64_t)i * no + q];
        ld4_add(sP + i * kNC, e, acc);
      }
#pragma unroll
      for (int w = 0; w < kNC; ++w)
        if (valid[w]) P.out[cell[w] * no + q] = acc[w];
    }
    __syncthreads();
  }
}

// indices of flagged cells, compacted on the device (order irrelevant: each
// cell is solved independently); idx[n] holds the count
__global__ void k_compact(const uint8_t* __restrict__ ood, int64_t n, int64_t* __restrict__ idx) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && ood[c]) {
    const unsigned long long k = atomicAdd(reinterpret_cast<unsigned long long*>(idx + n), 1ull);
    idx[k] = c;
  }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

// Band powers summed over cells, weighted: sum_c w_c out[c][b].  Lane b of a
// wave accumulates band b over the cells of its wave (one row read per cell,
// lanes on consecutive bands), the block's four waves are added in LDS, and
// a second kernel adds the blocks' partial sums in block order: the result
// does not depend on timing.
__global__ void __launch_bounds__(256) k_band_power_part(int nbd, int no, int64_t n, const double* __restrict__ out,
                                                        const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double s[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc = 0.0;
  if (lane < nbd)
    for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < n; c += (int64_t)gridDim.x * 4)
      acc += w[c] * out[c * no + lane];
  s[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) part[blockIdx.x * 64 + lane] = s[0][lane] + s[1][lane] + s[2][lane] + s[3][lane];
}

__global__ void k_band_power_sum(int nbd, const double* __restrict__ part, double* __restrict__ bp) {
  const int b = threadIdx.x;
  if (b >= nbd) return;
  double acc = 0.0;
  for (int k = 0; k < kBpBlocks; ++k) acc += part[k * 64 + b];
  bp[b] = acc;
}

size_t solve_lds(const pah_desc& d) {
  return sizeof(double) * (kNC * ((size_t)d.M + 3 * (size_t)d.n_lambda + 2 + kBk * kBk + kBk) +
                           2 * (size_t)d.M + d.n_lambda) +
         sizeof(int) * kNC;
}

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

struct pah_ctx {
  pah_desc d;
  PahLayout lay;
  unsigned char* tables = nullptr;
  bool built = false;
  int n_cu = 256;
  int blocks = 0;
  std::string err;
};

const pah_desc& pah_ctx_desc(const pah_ctx* c) { return c->d; }
const double* pah_ctx_dnu(const pah_ctx* c) {
  return c->built ? reinterpret_cast<const double*>(c->tables + c->lay.dnu) : nullptr;
}

namespace {
int32_t pfail(pah_ctx* c, int32_t code, const std::string& m) {
  if (c) c->err = m;
  return code;
}
const char* pcheck(const pah_desc* d) {
  if (!d) return "null descriptor";
  if (d->M < 3 || d->M > 4096) return "M must be in 3..4096";
  if (d->n_lambda < 2 || d->n_lambda > 4096) return "n_lambda must be in 2..4096";
  if (d->n_bands < 0 || d->n_bands > 64) return "n_bands must be in 0..64";
  if (!d->T || !d->U || !d->lambda_um || !d->cabs || !d->ccont || (d->n_bands > 0 && !d->cband))
    return "null device array";
  if (solve_lds(*d) > kMaxLds) return "M and n_lambda exceed the solver's LDS (6 M + 13 n_lambda <= 16246)";
  return nullptr;
}
int nblocks_of(int M) { return (M - 1 + kBk - 1) / kBk; }

// launch parameters shared by the exact solve and the fallback
SolveP solve_params(const pah_ctx* c) {
  const PahLayout& L = c->lay;
  const unsigned char* T = c->tables;
  SolveP P{};
  P.M = c->d.M; P.nl = c->d.n_lambda; P.nbd = c->d.n_bands; P.nblk = nblocks_of(c->d.M);
  P.cabs = c->d.cabs;
  P.U = c->d.U;
  P.E = reinterpret_cast<const double*>(T + L.E);
  P.fac = reinterpret_cast<const double*>(T + L.fac);
  P.invdu = reinterpret_cast<const double*>(T + L.invdu);
  P.mtab = reinterpret_cast<const uint32_t*>(T + L.mtab);
  P.adown = reinterpret_cast<const double*>(T + L.adown);
  P.em = reinterpret_cast<const double*>(T + L.em);
  return P;
}
}  // namespace

extern "C" {

int32_t pah_tables_bytes(const pah_desc* d, uint64_t* bytes) {
  if (pcheck(d) || !bytes) return MCRT_E_INVALID;
  *bytes = pah_layout(*d).total;
  return MCRT_OK;
}

int32_t pah_ctx_create(const pah_desc* d, pah_ctx** out) {
  if (!out) return MCRT_E_INVALID;
  *out = nullptr;
  if (pcheck(d)) return MCRT_E_INVALID;
  pah_ctx* c = new (std::nothrow) pah_ctx();
  if (!c) return MCRT_E_INVALID;
  c->d = *d;
  c->lay = pah_layout(*d);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    c->n_cu = ncu;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pah_solve, kThreads, solve_lds(*d)) !=
          hipSuccess || per_cu < 1)
    per_cu = 4;
  c->blocks = c->n_cu * per_cu;
  *out = c;
  return MCRT_OK;
}

void pah_ctx_destroy(pah_ctx* c) { delete c; }

const char* pah_last_error(const pah_ctx* c) { return c ? c->err.c_str() : "null context"; }

int32_t pah_build_tables(pah_ctx* c, void* tables, uint64_t bytes, hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!tables) return pfail(c, MCRT_E_INVALID, "null tables");
  if (bytes < c->lay.total) return pfail(c, MCRT_E_CAPACITY, "tables buffer too small");
  c->tables = static_cast<unsigned char*>(tables);
  const pah_desc& d = c->d;
  const PahLayout& L = c->lay;
  unsigned char* T = c->tables;
  auto D = [&](uint64_t o) { return reinterpret_cast<double*>(T + o); };
  const int M = d.M, nl = d.n_lambda;
  k_pah_bins<<<1, 256, 0, s>>>(nl, M, d.lambda_um, d.U, D(L.nu), D(L.dnu), D(L.ed), D(L.E),
                               D(L.fac), D(L.invdu));
  const int64_t mm = (int64_t)M * M;
  k_pah_m<<<(unsigned)((mm + 255) / 256), 256, 0, s>>>(M, nl, d.U, D(L.E),
                                                       reinterpret_cast<uint32_t*>(T + L.mtab));
  k_pah_em<<<M, 256, 0, s>>>(M, nl, d.n_bands, d.T, d.U, D(L.nu), D(L.dnu), d.cabs, d.cband, d.ccont,
                             D(L.adown), D(L.em));
  if (d.n_bands > 0) k_pah_bandw<<<d.n_bands, 256, 0, s>>>(nl, d.cband, D(L.dnu), D(L.bandw));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("pah table launch: ") + hipGetErrorString(e));
  c->built = true;
  return MCRT_OK;
}

int32_t pah_solve_exact(pah_ctx* c, const void* J, int32_t j_is_f32, int64_t n, double* out,
                        double* P_out, double* pabs_out, hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!c->built) return pfail(c, MCRT_E_STATE, "pah_solve_exact before pah_build_tables");
  if (n < 0) return pfail(c, MCRT_E_INVALID, "n < 0");
  if (n == 0) return MCRT_OK;
  if (!J || !out) return pfail(c, MCRT_E_INVALID, "null J or out");
  SolveP P = solve_params(c);
  P.j_f32 = j_is_f32 ? 1 : 0;
  P.n = n; P.J = J;
  P.out = out; P.P_out = P_out; P.pabs = pabs_out;
  const int64_t groups = (n + kNC - 1) / kNC;
  const int64_t blocks = groups < c->blocks ? groups : c->blocks;
  k_pah_solve<<<(unsigned)blocks, kThreads, solve_lds(c->d), s>>>(P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("pah solve launch: ") + hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_build_rows(pah_ctx* c, const double* out, int64_t n, double* rows, hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!c->built) return pfail(c, MCRT_E_STATE, "rows before pah_build_tables");
  if (n < 0) return pfail(c, MCRT_E_INVALID, "n < 0");
  if (n == 0) return MCRT_OK;
  if (!out || !rows) return pfail(c, MCRT_E_INVALID, "null out or rows");
  const size_t wbytes = sizeof(double) * (size_t)c->d.n_bands * c->d.n_lambda;
  const int in_lds = wbytes <= (size_t)kRowLdsMax ? 1 : 0;
  const int64_t want = (n + 3) / 4;
  const int64_t blocks = want < (int64_t)c->n_cu * 8 ? want : (int64_t)c->n_cu * 8;
  const double* wb = reinterpret_cast<const double*>(c->tables + c->lay.bandw);
  if (in_lds)
    k_pah_rows<true><<<(unsigned)blocks, 256, wbytes, s>>>(c->d.n_lambda, c->d.n_bands, n, out, wb, rows);
  else
    k_pah_rows<false><<<(unsigned)blocks, 256, 0, s>>>(c->d.n_lambda, c->d.n_bands, n, out, wb, rows);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("rows launch: ") + hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_band_power(pah_ctx* c, const double* out, int64_t n, const double* weight, double* bp_out,
                       hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!c->built) return pfail(c, MCRT_E_STATE, "band power before pah_build_tables");
  if (n < 0) return pfail(c, MCRT_E_INVALID, "n < 0");
  if (!out || !weight || !bp_out) return pfail(c, MCRT_E_INVALID, "null argument");
  if (c->d.n_bands == 0) return MCRT_OK;
  double* part = reinterpret_cast<double*>(c->tables + c->lay.bp_part);
  k_band_power_part<<<kBpBlocks, 256, 0, s>>>(c->d.n_bands, c->d.n_bands + c->d.n_lambda, n, out, weight, part);
  k_band_power_sum<<<1, 64, 0, s>>>(c->d.n_bands, part, bp_out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("band power launch: ") + hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_exact_fallback(pah_ctx* c, const float* J, int64_t n, const uint8_t* ood, double* out,
                           int64_t* idx, hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!c->built) return pfail(c, MCRT_E_STATE, "fallback before pah_build_tables");
  if (n < 0) return pfail(c, MCRT_E_INVALID, "n < 0");
  if (n == 0) return MCRT_OK;
  if (!J || !ood || !out || !idx) return pfail(c, MCRT_E_INVALID, "null argument");
  k_zero_i64<<<1, 1, 0, s>>>(idx + n);
  k_compact<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ood, n, idx);
  SolveP P = solve_params(c);
  P.j_f32 = 1;
  P.n = n; P.J = J;
  P.out = out;
  P.idx = idx;
  P.n_dev = idx + n;
  const int64_t groups = (n + kNC - 1) / kNC;
  const int64_t blocks = groups < c->blocks ? groups : c->blocks;
  k_pah_solve<<<(unsigned)blocks, kThreads, solve_lds(c->d), s>>>(P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("fallback launch: ") + hipGetErrorString(e));
  return MCRT_OK;
}

}  // extern "C"
