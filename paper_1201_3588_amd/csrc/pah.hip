// Exact steady-state temperature distribution P(T) of transiently heated PAHs
// and their band/continuum emission, per cell, in FP64 (paper Sec. 1, Sec. 4,
// Fig. 3: P(T) depends on the strength and the hardness of the field).
//
// P_f A_{f-1,f} = sum_{i<f} P_i B_{f,i},  B_{f,i} = sum_{k>=f} A_{k,i}.
// Forming B_{f,i} by running subtraction loses the hot tail to cancellation
// and storing it costs M^2/2 doubles per cell, so the f range is cut into
// blocks of kBk and every sum is kept positive:
//   pass 1 (top-down): D^b_i = sum_{k >= end of block b} A_{k,i}, per block,
//                      into a per-workgroup global scratch;
//   pass 2 (bottom-up, block b = [f_b, e_b)):
//     in_k  = sum_{i<f_b} P_i A_{k,i}  (k in the block),  Sin_f = sum_{k>=f} in_k
//     C0    = sum_{i<f_b} P_i D^b_i
//     Bin[f][i] = sum_{k=f}^{e_b-1} A_{k,i}  (f_b <= i < f < e_b)
//     P_f = (C0 + Sin_f + sum_{i=f_b}^{f-1} P_i (D^b_i + Bin[f][i])) / A_{f-1,f}.
// Four cells per 256-thread workgroup (persistent grid): each cell-independent
// table entry is loaded once for the four cells, and the in-block recurrence
// of cell w runs on wave w with shuffle reductions.
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

struct PahLayout {
  uint64_t nu, dnu, ed, Elo, Ehi, Ue, wup, jb, wtop, jlim, adown, em, bandw, total;
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
  L.Elo = take(8 * nl);
  L.Ehi = take(8 * nl);
  L.Ue = take(8 * (M + 1));
  L.wup = take(8 * M * M);
  L.jb = take(2 * M * M);
  L.wtop = take(8 * M * nl);
  L.jlim = take(4 * M);
  L.adown = take(8 * M);
  L.em = take(8 * M * no);
  L.bandw = take(8 * (uint64_t)(d.n_bands > 0 ? d.n_bands : 1) * nl);
  L.total = off;
  return L;
}

// wavelength bins: centres, widths, ascending edges (micron), photon-energy edges
__global__ void k_pah_bins(int nl, int M, const double* __restrict__ lam, const double* __restrict__ U,
                           double* nu, double* dnu, double* ed, double* Elo, double* Ehi, double* Ue) {
  for (int j = threadIdx.x; j <= nl; j += blockDim.x) {
    double e;
    if (j == 0) e = lam[0] * lam[0] / sqrt(lam[0] * lam[1]);
    else if (j == nl) e = lam[nl - 1] * lam[nl - 1] / sqrt(lam[nl - 2] * lam[nl - 1]);
    else e = sqrt(lam[j - 1] * lam[j]);
    ed[j] = e;
  }
  for (int i = threadIdx.x; i <= M; i += blockDim.x) {
    if (i == 0) Ue[0] = U[0];
    else if (i == M) Ue[M] = U[M - 1] + 0.5 * (U[M - 1] - U[M - 2]);
    else Ue[i] = 0.5 * (U[i - 1] + U[i]);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    nu[j] = kC / (lam[j] * 1e-4);
    dnu[j] = kC / (ed[j] * 1e-4) - kC / (ed[j + 1] * 1e-4);
    Ehi[j] = kH * kC / (ed[j] * 1e-4);
    Elo[j] = kH * kC / (ed[j + 1] * 1e-4);
  }
}

// heating weight and wavelength bin of every jump i -> k (k < M-1)
__global__ void k_pah_up(int M, int nl, const double* __restrict__ U, const double* __restrict__ Ue,
                         const double* __restrict__ ed, double* __restrict__ wup,
                         uint16_t* __restrict__ jb) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * M) return;
  const int k = (int)(q / M), i = (int)(q % M);
  double w = 0.0;
  int bin = 0;
  if (i < k && k < M - 1) {
    const double E = U[k] - U[i];
    const double lam = kH * kC / E * 1e4;   // micron
    if (lam >= ed[0] && lam < ed[nl]) {
      int lo = 0, hi = nl - 1;              // largest j with ed[j] <= lam
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ed[mid] <= lam) lo = mid; else hi = mid - 1;
      }
      bin = lo;
      w = (Ue[k + 1] - Ue[k]) * 4.0 * kPi / (kH * E);
    }
  }
  wup[q] = w;
  jb[q] = (uint16_t)bin;
}

// number of leading wavelength bins that reach the top bin from state i
// (photon energy falls with the bin index, so the overlapping bins lead)
__global__ void k_pah_jlim(int M, int nl, const double* __restrict__ wtop, int* __restrict__ jlim) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int last = 0;
  for (int j = 0; j < nl; ++j)
    if (wtop[(int64_t)i * nl + j] != 0.0) last = j + 1;
  jlim[i] = last;
}

// top bin: integral over every jump at or above its lower edge
__global__ void k_pah_top(int M, int nl, const double* __restrict__ U, const double* __restrict__ Ue,
                          const double* __restrict__ Elo, const double* __restrict__ Ehi,
                          double* __restrict__ wtop) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * nl) return;
  const int i = (int)(q / nl), j = (int)(q % nl);
  double w = 0.0;
  if (i < M - 1) {
    const double Emin = Ue[M - 1] - U[i];
    const double a = Elo[j] > Emin ? Elo[j] : Emin;
    if (Ehi[j] > a) w = 4.0 * kPi / kH * log(Ehi[j] / a);
  }
  wtop[q] = w;
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
// spread by their profiles, running sum normalised to end at exactly 1
__global__ void __launch_bounds__(256) k_pah_rows(int nl, int nbd, int64_t n, const double* __restrict__ out,
                                                  const double* __restrict__ w, double* __restrict__ rows) {
  extern __shared__ double sc[];                 // [nl] scan buffer
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  const int no = nbd + nl;
  const double* o = out + c * no;
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    double e = o[nbd + j];
    for (int b = 0; b < nbd; ++b) e += o[b] * w[(int64_t)b * nl + j];
    sc[j] = e;
  }
  __syncthreads();
  // inclusive scan (Hillis-Steele) over nl entries
  for (int off = 1; off < nl; off <<= 1) {
    double v[16];
    int cnt = 0;
    for (int j = threadIdx.x; j < nl; j += blockDim.x) v[cnt++] = j >= off ? sc[j - off] : 0.0;
    __syncthreads();
    cnt = 0;
    for (int j = threadIdx.x; j < nl; j += blockDim.x) sc[j] += v[cnt++];
    __syncthreads();
  }
  const double tot = sc[nl - 1];
  for (int j = threadIdx.x; j < nl; j += blockDim.x)
    rows[c * nl + j] = (j == nl - 1 || !(tot > 0.0)) ? 1.0 : sc[j] / tot;
}

struct SolveP {
  int M, nl, nbd, nblk, j_f32;
  int64_t n;
  const void* J;
  const double* cabs;
  const double* dnu;
  const double* wup;
  const uint16_t* jb;
  const double* wtop;
  const int* jlim;
  const double* adown;
  const double* em;
  double* out;
  double* P_out;
  double* pabs;
  double* ws;
  const int64_t* idx;     // cells to solve (null: 0..n-1)
  const int64_t* n_dev;   // device count of idx (null: n)
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// sums of kNC per-thread values over the workgroup; every thread gets all
// kNC results in out[]
__device__ __forceinline__ void block_sum_nc(const double* v, double* red, double* out) {
  const int w = threadIdx.x >> 6;
  double x[kNC];
#pragma unroll
  for (int c = 0; c < kNC; ++c) x[c] = wave_sum_d(v[c]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < kNC; ++c) red[w * kNC + c] = x[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kNC; ++c) {
    double s = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) s += red[k * kNC + c];
    out[c] = s;
  }
}

// kNC cells per workgroup: every cell-independent table entry is loaded once
// and applied to kNC cells; the in-block recurrence of cell w runs on wave w.
__global__ void __launch_bounds__(kThreads) k_pah_solve(const SolveP P) {
  extern __shared__ double sm[];
  const int M = P.M, nl = P.nl, nbd = P.nbd, nblk = P.nblk;
  const int no = nbd + nl;
  double* sP = sm;                              // [kNC][M]
  double* sTop = sP + kNC * M;                  // [kNC][M]
  double* sCJ = sTop + kNC * M;                 // [kNC][nl]
  double* sBin = sCJ + kNC * nl;                // [kNC][kBk * kBk]
  double* sIn = sBin + kNC * kBk * kBk;         // [kNC][kBk]
  double* red = sIn + kNC * kBk;                // [4 * kNC]
  int* sScale = reinterpret_cast<int*>(red + 4 * kNC);   // [kNC]
  double* D = P.ws + (int64_t)blockIdx.x * kNC * nblk * M;    // [kNC][nblk][M]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const double fourpi_h = 4.0 * kPi / kH;
  (void)fourpi_h;

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
    // ---- field times cross-section; absorbed power (wave w: cell w)
    for (int q = t; q < kNC * nl; q += kThreads) {
      const int w = q / nl, j = q % nl;
      double Jj = 0.0;
      if (valid[w])
        Jj = P.j_f32 ? (double)reinterpret_cast<const float*>(P.J)[cell[w] * nl + j]
                     : reinterpret_cast<const double*>(P.J)[cell[w] * nl + j];
      sCJ[w * nl + j] = P.cabs[j] * Jj;
    }
    __syncthreads();
    {
      double pa = 0.0;
      for (int j = lane; j < nl; j += 64) pa += sCJ[wave * nl + j] * P.dnu[j];
      pa = wave_sum_d(pa);
      if (wave < kNC && lane == 0 && P.pabs && valid[wave]) P.pabs[cell[wave]] = 4.0 * kPi * pa;
    }
    // ---- top-bin rates (only the leading bins overlap)
    for (int i = t; i < M; i += kThreads) {
      double acc[kNC] = {};
      const double* wt = P.wtop + (int64_t)i * nl;
      const int jl = P.jlim[i];
      for (int j = 0; j < jl; ++j) {
        const double a = wt[j];
#pragma unroll
        for (int w = 0; w < kNC; ++w) acc[w] += a * sCJ[w * nl + j];
      }
#pragma unroll
      for (int w = 0; w < kNC; ++w) sTop[w * M + i] = acc[w];
    }
    __syncthreads();

    // ---- pass 1: D^b_i for every cell, columns paired (i, M-1-i)
    for (int h = t; h < (M + 1) / 2; h += kThreads) {
      for (int side = 0; side < 2; ++side) {
        const int i = side == 0 ? h : M - 1 - h;
        if (side == 1 && i == h) break;
        double S[kNC] = {};
#pragma unroll
        for (int w = 0; w < kNC; ++w) D[((int64_t)w * nblk + nblk - 1) * M + i] = 0.0;
        for (int k = M - 1; k > i; --k) {
          if (k == M - 1) {
#pragma unroll
            for (int w = 0; w < kNC; ++w) S[w] += sTop[w * M + i];
          } else {
            const int64_t q = (int64_t)k * M + i;
            const double a = P.wup[q];
            const int jj = P.jb[q];
#pragma unroll
            for (int w = 0; w < kNC; ++w) S[w] += a * sCJ[w * nl + jj];
          }
          if (k > kBk && ((k - 1) % kBk) == 0) {
            const int b = (k - 1) / kBk - 1;
#pragma unroll
            for (int w = 0; w < kNC; ++w) D[((int64_t)w * nblk + b) * M + i] = S[w];
          }
        }
      }
    }
    if (t < kNC) { sP[t * M] = 1.0; sScale[t] = 0; }
    __syncthreads();

    // ---- pass 2: blocks of f upward
    for (int b = 0; b < nblk; ++b) {
      const int fb = 1 + kBk * b;
      const int eb = fb + kBk < M ? fb + kBk : M;
      const int bk = eb - fb;
      // in_k for k in the block: 32 k-slots x 8 i-groups, all cells per load
      {
        const int kk = t >> 3, g = t & 7;
        double acc[kNC] = {};
        if (kk < bk) {
          const int k = fb + kk;
          if (k == M - 1) {
            for (int i = g; i < fb; i += 8)
#pragma unroll
              for (int w = 0; w < kNC; ++w) acc[w] += sP[w * M + i] * sTop[w * M + i];
          } else {
            for (int i = g; i < fb; i += 8) {
              const int64_t q = (int64_t)k * M + i;
              const double a = P.wup[q];
              const int jj = P.jb[q];
#pragma unroll
              for (int w = 0; w < kNC; ++w) acc[w] += sP[w * M + i] * (a * sCJ[w * nl + jj]);
            }
          }
        }
#pragma unroll
        for (int w = 0; w < kNC; ++w) {
          acc[w] += __shfl_xor(acc[w], 1);
          acc[w] += __shfl_xor(acc[w], 2);
          acc[w] += __shfl_xor(acc[w], 4);
          if (g == 0 && kk < kBk) sIn[w * kBk + kk] = kk < bk ? acc[w] : 0.0;
        }
      }
      // C0 = sum_{i<fb} P_i D^b_i, per cell
      double C0[kNC];
      {
        double v[kNC] = {};
        for (int i = t; i < fb; i += kThreads)
#pragma unroll
          for (int w = 0; w < kNC; ++w) v[w] += sP[w * M + i] * D[((int64_t)w * nblk + b) * M + i];
        block_sum_nc(v, red, C0);
      }
      // Bin[f][i] = sum_{k=f}^{eb-1} A_{k,i}: thread (w, column)
      if (t < kNC * kBk) {
        const int w = t / kBk, col = t % kBk;
        if (col < bk) {
          const int i = fb + col;
          double acc = 0.0;
          for (int k = eb - 1; k > i; --k) {
            if (k == M - 1) acc += sTop[w * M + i];
            else {
              const int64_t q = (int64_t)k * M + i;
              acc += P.wup[q] * sCJ[w * nl + P.jb[q]];
            }
            sBin[w * kBk * kBk + (k - fb) * kBk + col] = acc;
          }
        }
      }
      __syncthreads();
      if (t < kNC) {                       // suffix sums of in_k
        double acc = 0.0;
        for (int kk = bk - 1; kk >= 0; --kk) { acc += sIn[t * kBk + kk]; sIn[t * kBk + kk] = acc; }
      }
      __syncthreads();
      // sequential recurrence: wave w for cell w; lane l holds P_{fb+l}
      if (wave < kNC) {
        const int w = wave;
        const double* Db = D + ((int64_t)w * nblk + b) * M;
        const double Dl = lane < bk ? Db[fb + lane] : 0.0;
        const double* bin = sBin + w * kBk * kBk;
        const double* sin_ = sIn + w * kBk;
        double myP = 0.0;
        int nsc = 0;                       // rescales by 2^-664 inside this block
        double c0 = C0[w];
        for (int fl = 0; fl < bk; ++fl) {
          const int f = fb + fl;
          const double term = lane < fl ? myP * (Dl + bin[fl * kBk + lane]) : 0.0;
          const double s = wave_sum_d(term);
          const double sin_f = nsc ? ldexp(sin_[fl], -664 * nsc) : sin_[fl];
          const double Pf = (c0 + sin_f + s) / P.adown[f];
          if (lane == fl) myP = Pf;
          if (Pf > 1e200) {                 // keep the unnormalised P finite
            ++nsc;
            if (lane <= fl) myP = ldexp(myP, -664);
            c0 = ldexp(c0, -664);
          }
        }
        if (lane < bk) sP[w * M + fb + lane] = myP;
        if (lane == 0) sScale[w] = nsc;
      }
      __syncthreads();
      for (int q = t; q < kNC * fb; q += kThreads) {
        const int w = q / fb, i = q % fb;
        const int nsc = sScale[w];
        if (nsc) sP[w * M + i] = ldexp(sP[w * M + i], -664 * nsc);
      }
      __syncthreads();
    }

    // ---- normalise (wave w: cell w) and emit
    if (wave < kNC) {
      double tot = 0.0;
      for (int i = lane; i < M; i += 64) tot += sP[wave * M + i];
      tot = wave_sum_d(tot);
      for (int i = lane; i < M; i += 64) sP[wave * M + i] /= tot;
    }
    __syncthreads();
    if (P.P_out)
      for (int q = t; q < kNC * M; q += kThreads) {
        const int w = q / M, i = q % M;
        if (valid[w]) P.P_out[cell[w] * M + i] = sP[w * M + i];
      }
    for (int q = t; q < no; q += kThreads) {
      double acc[kNC] = {};
      for (int i = 1; i < M; ++i) {
        const double e = P.em[(int64_t)i * no + q];
#pragma unroll
        for (int w = 0; w < kNC; ++w) acc[w] += sP[w * M + i] * e;
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

size_t solve_lds(const pah_desc& d) {
  return sizeof(double) * (kNC * (2 * (size_t)d.M + d.n_lambda + kBk * kBk + kBk) + 4 * kNC) +
         sizeof(int) * kNC + 16;
}

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
  return nullptr;
}
int nblocks_of(int M) { return (M - 1 + kBk - 1) / kBk; }
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
  k_pah_bins<<<1, 256, 0, s>>>(nl, M, d.lambda_um, d.U, D(L.nu), D(L.dnu), D(L.ed), D(L.Elo),
                               D(L.Ehi), D(L.Ue));
  const int64_t mm = (int64_t)M * M;
  k_pah_up<<<(unsigned)((mm + 255) / 256), 256, 0, s>>>(M, nl, d.U, D(L.Ue), D(L.ed), D(L.wup),
                                                        reinterpret_cast<uint16_t*>(T + L.jb));
  const int64_t ml = (int64_t)M * nl;
  k_pah_top<<<(unsigned)((ml + 255) / 256), 256, 0, s>>>(M, nl, d.U, D(L.Ue), D(L.Elo), D(L.Ehi),
                                                         D(L.wtop));
  k_pah_jlim<<<(M + 255) / 256, 256, 0, s>>>(M, nl, D(L.wtop), reinterpret_cast<int*>(T + L.jlim));
  k_pah_em<<<M, 256, 0, s>>>(M, nl, d.n_bands, d.T, d.U, D(L.nu), D(L.dnu), d.cabs, d.cband, d.ccont,
                             D(L.adown), D(L.em));
  if (d.n_bands > 0) k_pah_bandw<<<d.n_bands, 256, 0, s>>>(nl, d.cband, D(L.dnu), D(L.bandw));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("pah table launch: ") + hipGetErrorString(e));
  c->built = true;
  return MCRT_OK;
}

int32_t pah_workspace_bytes(const pah_ctx* c, uint64_t* bytes) {
  if (!c || !bytes) return MCRT_E_INVALID;
  *bytes = (uint64_t)c->blocks * kNC * nblocks_of(c->d.M) * c->d.M * sizeof(double);
  return MCRT_OK;
}

int32_t pah_solve_exact(pah_ctx* c, const void* J, int32_t j_is_f32, int64_t n, double* out,
                        double* P_out, double* pabs_out, void* ws, uint64_t ws_bytes, hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!c->built) return pfail(c, MCRT_E_STATE, "pah_solve_exact before pah_build_tables");
  if (n < 0) return pfail(c, MCRT_E_INVALID, "n < 0");
  if (n == 0) return MCRT_OK;
  if (!J || !out || !ws) return pfail(c, MCRT_E_INVALID, "null J, out or workspace");
  uint64_t need = 0;
  pah_workspace_bytes(c, &need);
  if (ws_bytes < need) return pfail(c, MCRT_E_CAPACITY, "workspace too small");
  const PahLayout& L = c->lay;
  unsigned char* T = c->tables;
  SolveP P{};
  P.M = c->d.M; P.nl = c->d.n_lambda; P.nbd = c->d.n_bands; P.nblk = nblocks_of(c->d.M);
  P.j_f32 = j_is_f32 ? 1 : 0;
  P.n = n; P.J = J; P.cabs = c->d.cabs;
  P.dnu = reinterpret_cast<const double*>(T + L.dnu);
  P.wup = reinterpret_cast<const double*>(T + L.wup);
  P.jb = reinterpret_cast<const uint16_t*>(T + L.jb);
  P.wtop = reinterpret_cast<const double*>(T + L.wtop);
  P.jlim = reinterpret_cast<const int*>(T + L.jlim);
  P.adown = reinterpret_cast<const double*>(T + L.adown);
  P.em = reinterpret_cast<const double*>(T + L.em);
  P.out = out; P.P_out = P_out; P.pabs = pabs_out;
  P.ws = static_cast<double*>(ws);
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
  if (c->d.n_lambda > 16 * 256) return pfail(c, MCRT_E_UNSUPPORTED, "n_lambda > 4096");
  k_pah_rows<<<(unsigned)n, 256, sizeof(double) * c->d.n_lambda, s>>>(
      c->d.n_lambda, c->d.n_bands, n, out, reinterpret_cast<const double*>(c->tables + c->lay.bandw), rows);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(c, MCRT_E_HIP, std::string("rows launch: ") + hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_exact_fallback(pah_ctx* c, const float* J, int64_t n, const uint8_t* ood, double* out,
                           int64_t* idx, void* ws, uint64_t ws_bytes, hipStream_t s) {
  if (!c) return MCRT_E_INVALID;
  if (!c->built) return pfail(c, MCRT_E_STATE, "fallback before pah_build_tables");
  if (n < 0) return pfail(c, MCRT_E_INVALID, "n < 0");
  if (n == 0) return MCRT_OK;
  if (!J || !ood || !out || !idx || !ws) return pfail(c, MCRT_E_INVALID, "null argument");
  uint64_t need = 0;
  pah_workspace_bytes(c, &need);
  if (ws_bytes < need) return pfail(c, MCRT_E_CAPACITY, "workspace too small");
  k_zero_i64<<<1, 1, 0, s>>>(idx + n);
  k_compact<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ood, n, idx);
  const PahLayout& L = c->lay;
  unsigned char* T = c->tables;
  SolveP P{};
  P.M = c->d.M; P.nl = c->d.n_lambda; P.nbd = c->d.n_bands; P.nblk = nblocks_of(c->d.M);
  P.j_f32 = 1;
  P.n = n; P.J = J; P.cabs = c->d.cabs;
  P.dnu = reinterpret_cast<const double*>(T + L.dnu);
  P.wup = reinterpret_cast<const double*>(T + L.wup);
  P.jb = reinterpret_cast<const uint16_t*>(T + L.jb);
  P.wtop = reinterpret_cast<const double*>(T + L.wtop);
  P.jlim = reinterpret_cast<const int*>(T + L.jlim);
  P.adown = reinterpret_cast<const double*>(T + L.adown);
  P.em = reinterpret_cast<const double*>(T + L.em);
  P.out = out;
  P.ws = static_cast<double*>(ws);
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
