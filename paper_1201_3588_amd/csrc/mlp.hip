// PAH emission surrogate: a 3-layer perceptron (n_in -> n_h -> n_h -> n_out,
// SiLU) trained on cells that the exact P(T) solver has solved.  Products run
// on the CDNA4 matrix cores (v_mfma_f32_32x32x16_bf16: bfloat16 operands,
// FP32 accumulation); weights keep FP32 masters updated by Adam and bfloat16
// working copies; the tile loader reads either operand layout, so one
// bfloat16 copy of each weight matrix serves forward and backward products.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "mcrt_internal.h"
#include "pah.h"
#include "pah_internal.h"

using namespace mcrt;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

enum { EPI_F32 = 0, EPI_SILU = 1, EPI_DSILU = 2 };

// C[m][n] = sum_k A(m,k) B(k,n); A(m,k) = ta ? A[k*lda+m] : A[m*lda+k];
// B(k,n) = tb ? B[n*ldb+k] : B[k*ldb+n].  bfloat16 operands (as uint16).
struct GemmP {
  int M, N, K, lda, ldb, ta, tb;
  const uint16_t* A;
  const uint16_t* B;
  const float* bias;    // [N] or null
  float* C;             // EPI_F32: [M][ldc]; EPI_SILU: pre-activation out (or null)
  int ldc;
  uint16_t* H;          // EPI_SILU: bf16 activation; EPI_DSILU: bf16 gradient
  int ldh;
  const float* Z;       // EPI_DSILU: stored pre-activation [M][ldz]
  int ldz;
  int kchunk;           // EPI_F32 split over K: blockIdx.z takes [z kchunk, (z+1) kchunk)
  float* part;          // and writes its partial product to part[z][M][N] (null: no split)
  int va, vb;           // A, B allow 16-byte loads (16-byte aligned base, ld a multiple of 8)
};

constexpr int BM = 64, BN = 64, BK = 32, PADK = 40;

// 64 x 32 tile of X(r, k) (r = row of the tile, k contiguous in LDS).  Each
// thread reads 8 consecutive elements: one 16-byte load where the operand
// allows it (vec) and the 8 lie inside it, else element by element with
// zeros outside (the same values either way).
__device__ __forceinline__ void load_tile(uint16_t (*S)[PADK], const uint16_t* __restrict__ G, int ld,
                                          bool kmajor, int r0, int k0, int R, int K, bool vec) {
  const int t = threadIdx.x;
  if (!kmajor) {                 // G[r*ld + k]: 8 consecutive k per thread
    const int r = t >> 2, kc = (t & 3) * 8;
    const int gr = r0 + r;
    if (vec && gr < R && k0 + kc + 8 <= K) {
      *reinterpret_cast<u16x8*>(&S[r][kc]) = *reinterpret_cast<const u16x8*>(G + (int64_t)gr * ld + k0 + kc);
      return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int gk = k0 + kc + i;
      S[r][kc + i] = (gr < R && gk < K) ? G[(int64_t)gr * ld + gk] : (uint16_t)0;
    }
  } else {                       // G[k*ld + r]: 8 consecutive r per thread
    const int kr = t >> 3, rc = (t & 7) * 8;
    const int gk = k0 + kr;
    if (vec && gk < K && r0 + rc + 8 <= R) {
      const u16x8 v = *reinterpret_cast<const u16x8*>(G + (int64_t)gk * ld + r0 + rc);
#pragma unroll
      for (int i = 0; i < 8; ++i) S[rc + i][kr] = v[i];
      return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int gr = r0 + rc + i;
      S[rc + i][kr] = (gr < R && gk < K) ? G[(int64_t)gk * ld + gr] : (uint16_t)0;
    }
  }
}

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(const GemmP p) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][PADK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][PADK];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool split = EPI == EPI_F32 && p.part != nullptr;
  const int kbeg = split ? (int)blockIdx.z * p.kchunk : 0;
  const int kend = split ? min(p.K, kbeg + p.kchunk) : p.K;
  f32x16 acc = {};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    load_tile(As, p.A, p.lda, p.ta != 0, m0, k0, p.M, kend, p.va != 0);
    load_tile(Bs, p.B, p.ldb, p.tb == 0, n0, k0, p.N, kend, p.vb != 0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const u16x8 a = *reinterpret_cast<const u16x8*>(&As[wm + (lane & 31)][kk + 8 * (lane >> 5)]);
      const u16x8 b = *reinterpret_cast<const u16x8*>(&Bs[wn + (lane & 31)][kk + 8 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element r of lane l: row 8*(r/4) + 4*(l/32) + r%4, column l%32
  const int col = n0 + wn + (lane & 31);
  if (col >= p.N) return;
  const float bcol = p.bias ? p.bias[col] : 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row >= p.M) continue;
    const float v = acc[r] + bcol;
    if (EPI == EPI_F32) {
      if (split) p.part[((int64_t)blockIdx.z * p.M + row) * p.N + col] = acc[r];
      else p.C[(int64_t)row * p.ldc + col] = v;
    } else if (EPI == EPI_SILU) {
      if (p.C) p.C[(int64_t)row * p.ldc + col] = v;
      p.H[(int64_t)row * p.ldh + col] = f2bf(silu(v));
    } else {
      p.H[(int64_t)row * p.ldh + col] = f2bf(v * dsilu(p.Z[(int64_t)row * p.ldz + col]));
    }
  }
}

// an operand allows 16-byte loads of 8 consecutive elements
bool vec_ok(const uint16_t* G, int ld) { return ld % 8 == 0 && (reinterpret_cast<uintptr_t>(G) & 15u) == 0; }

template <int EPI>
hipError_t gemm(GemmP p, hipStream_t s) {
  p.va = vec_ok(p.A, p.lda);
  p.vb = vec_ok(p.B, p.ldb);
  dim3 grid((p.N + BN - 1) / BN, (p.M + BM - 1) / BM);
  k_gemm<EPI><<<grid, 256, 0, s>>>(p);
  return hipGetLastError();
}

// C = sum over the splits of part[z], in split order (deterministic)
__global__ void k_split_sum(const float* __restrict__ part, int ks, int M, int N, float* __restrict__ C, int ldc) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * N) return;
  float acc = 0.0f;
  for (int z = 0; z < ks; ++z) acc += part[(int64_t)z * M * N + q];
  C[(q / N) * ldc + q % N] = acc;
}

constexpr int kMaxSplit = 16;

// weight gradients: few output tiles and a long K (the batch), so K is split
// until the grid covers the chip; partial tiles go to `part`, then are summed
hipError_t gemm_f32_split(GemmP p, float* part, hipStream_t s) {
  const int tiles = ((p.N + BN - 1) / BN) * ((p.M + BM - 1) / BM);
  int ks = 1;
  while (ks < kMaxSplit && tiles * ks < 256 && p.K / (2 * ks) >= 4 * BK) ks *= 2;
  if (ks == 1) return gemm<EPI_F32>(p, s);
  p.kchunk = ((p.K + ks - 1) / ks + BK - 1) / BK * BK;
  ks = (p.K + p.kchunk - 1) / p.kchunk;
  p.part = part;
  p.va = vec_ok(p.A, p.lda);
  p.vb = vec_ok(p.B, p.ldb);
  dim3 grid((p.N + BN - 1) / BN, (p.M + BM - 1) / BM, ks);
  k_gemm<EPI_F32><<<grid, 256, 0, s>>>(p);
  const int64_t mn = (int64_t)p.M * p.N;
  k_split_sum<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(part, ks, p.M, p.N, p.C, p.ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
struct MlpLayout {
  // fp32 parameter block [W1 b1 W2 b2 W3 b3] and three blocks like it
  uint64_t params, grads, adam_m, adam_v, n_params;
  uint64_t oW1, ob1, oW2, ob2, oW3, ob3;     // element offsets inside a block
  uint64_t W1h, W2h, W3h;                    // bf16 copies
  uint64_t x_mu, x_sd, x_lo, x_hi, y_mu, y_sd;
  uint64_t X16, Z1, H1, Z2, H2, Y, dY16, dZ2, dZ1, loss, Wpk, part, total;
};

MlpLayout mlp_layout(int ni, int nh, int no, int batch) {
  MlpLayout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t b) {
    const uint64_t o = off;
    off += (b + 255) & ~uint64_t(255);
    return o;
  };
  L.oW1 = 0;
  L.ob1 = L.oW1 + (uint64_t)nh * ni;
  L.oW2 = L.ob1 + nh;
  L.ob2 = L.oW2 + (uint64_t)nh * nh;
  L.oW3 = L.ob2 + nh;
  L.ob3 = L.oW3 + (uint64_t)no * nh;
  L.n_params = L.ob3 + no;
  L.params = take(4 * L.n_params);
  L.grads = take(4 * L.n_params);
  L.adam_m = take(4 * L.n_params);
  L.adam_v = take(4 * L.n_params);
  L.W1h = take(2ull * nh * ni);
  L.W2h = take(2ull * nh * nh);
  L.W3h = take(2ull * no * nh);
  L.x_mu = take(4ull * ni);
  L.x_sd = take(4ull * ni);
  L.x_lo = take(4ull * ni);
  L.x_hi = take(4ull * ni);
  L.y_mu = take(4ull * no);
  L.y_sd = take(4ull * no);
  const uint64_t B = (uint64_t)batch;
  L.X16 = take(2 * B * ni);
  L.Z1 = take(4 * B * nh);
  L.H1 = take(2 * B * nh);
  L.Z2 = take(4 * B * nh);
  L.H2 = take(2 * B * nh);
  L.Y = take(4 * B * no);
  L.dY16 = take(2 * B * no);
  L.dZ2 = take(2 * B * nh);
  L.dZ1 = take(2 * B * nh);
  L.loss = take(256);
  L.Wpk = take(2ull * 3 * 256 * 256);
  {
    uint64_t mx = (uint64_t)no * nh;
    if ((uint64_t)nh * nh > mx) mx = (uint64_t)nh * nh;
    if ((uint64_t)nh * ni > mx) mx = (uint64_t)nh * ni;
    L.part = take(4ull * kMaxSplit * mx);      // split-K partial products
  }
  L.total = off;
  return L;
}

__global__ void k_to_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// bf16 working copy of one weight matrix
__global__ void k_refresh(const float* __restrict__ W, int64_t n, uint16_t* __restrict__ Wh) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) Wh[q] = f2bf(W[q]);
}

// dY = 2 (Y - T) / (n n_out) in bf16, and the loss sum
__global__ void k_loss(const float* __restrict__ Y, const float* __restrict__ T, int64_t n, int no,
                       uint16_t* __restrict__ dY, float* loss) {
  __shared__ float red[256];
  const int64_t N = n * no;
  const float sc = 2.0f / (float)N;
  float acc = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    acc += d * d;
    dY[i] = f2bf(sc * d);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] / (float)N);
}

// column sums of a bf16 [n][N] matrix: a strip of 64 columns per workgroup,
// 16 row groups with 4 independent accumulators each, combined in LDS in a
// fixed order (deterministic)
constexpr int kColRows = 16;
__global__ void __launch_bounds__(64 * kColRows) k_colsum(const uint16_t* __restrict__ G, int64_t n, int N,
                                                          float* __restrict__ out) {
  __shared__ float part[kColRows][64];
  const int lc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lc;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  if (c < N) {
    int64_t r = rg;
    for (; r + 3 * kColRows < n; r += 4 * kColRows) {
      a0 += bf2f(G[r * N + c]);
      a1 += bf2f(G[(r + kColRows) * N + c]);
      a2 += bf2f(G[(r + 2 * kColRows) * N + c]);
      a3 += bf2f(G[(r + 3 * kColRows) * N + c]);
    }
    for (; r < n; r += kColRows) a0 += bf2f(G[r * N + c]);
  }
  part[rg][lc] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (rg == 0 && c < N) {
    float s = 0.0f;
    for (int k = 0; k < kColRows; ++k) s += part[k][lc];
    out[c] = s;
  }
}

// Adam (Kingma & Ba 2015) on the FP32 masters, bias-corrected with step t
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// network inputs of one cell: the share of the absorbed power in each
// wavelength bin, f_j = C_j J_j dnu_j / sum_j' C J dnu (the emission per
// absorbed power is linear in these while single photons heat the molecule),
// then log10 of the absorbed power 4 pi sum C J dnu (the field strength, which
// governs multi-photon heating).  Returns the absorbed power.
__device__ __forceinline__ double cell_features(const float* __restrict__ Jc, int nl,
                                                const double* __restrict__ cabs,
                                                const double* __restrict__ dnu, float* x) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < nl; j += blockDim.x) s += cabs[j] * (double)Jc[j] * dnu[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double tot = red[0];
  __syncthreads();
  const double inv = tot > 0.0 ? 1.0 / tot : 0.0;
  for (int j = threadIdx.x; j < nl; j += blockDim.x) x[j] = (float)(cabs[j] * (double)Jc[j] * dnu[j] * inv);
  const double pabs = 4.0 * kPi * tot;
  if (threadIdx.x == 0) x[nl] = (float)log10(fmax(pabs, 1e-300));
  return pabs;
}

// inference input: standardised features in bf16, absorbed power, range flag
__global__ void k_mlp_in(const float* __restrict__ J, int64_t n, int nl, const double* __restrict__ cabs,
                         const double* __restrict__ dnu, const float* __restrict__ mu,
                         const float* __restrict__ sd, const float* __restrict__ lo,
                         const float* __restrict__ hi, float margin, uint16_t* __restrict__ X,
                         double* __restrict__ pabs, uint8_t* __restrict__ ood) {
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  extern __shared__ float xs[];                 // [nl + 1]
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  const double pa = cell_features(J + c * nl, nl, cabs, dnu, xs);
  __syncthreads();
  const int ni = nl + 1;
  for (int j = threadIdx.x; j < ni; j += blockDim.x) {
    const float x = (xs[j] - mu[j]) / sd[j];
    if (x < lo[j] - margin || x > hi[j] + margin) bad = 1;
    X[c * ni + j] = f2bf(x);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pabs[c] = pa;
    ood[c] = (bad && pa > 0.0) ? 1 : 0;     // a dark cell's answer is exact: F = 0
  }
}

// inference output: F = 10^(y sd + mu) P_abs, energy-balance flag
__global__ void k_mlp_out(const float* __restrict__ Y, int64_t n, int no, const float* __restrict__ mu,
                          const float* __restrict__ sd, const double* __restrict__ pabs, float tol,
                          double* __restrict__ out, uint8_t* __restrict__ ood) {
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  __shared__ double red[256];
  double s = 0.0;
  for (int q = threadIdx.x; q < no; q += blockDim.x) {
    const double f = pabs[c] > 0.0 ? (double)exp10f(Y[c * no + q] * sd[q] + mu[q]) * pabs[c] : 0.0;
    out[c * no + q] = f;
    s += f;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(fabs(red[0] - pabs[c]) <= tol * pabs[c])) ood[c] |= 2;
}

// training pairs: x = cell features, y = log10(F / P_abs) (floored), as floats
__global__ void k_prep(const float* __restrict__ J, const double* __restrict__ out,
                       const double* __restrict__ pabs, int64_t n, int nl, int no,
                       const double* __restrict__ cabs, const double* __restrict__ dnu,
                       float* __restrict__ X, float* __restrict__ Y) {
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  cell_features(J + c * nl, nl, cabs, dnu, X + c * (nl + 1));
  const double pa = pabs[c];
  for (int q = threadIdx.x; q < no; q += blockDim.x)
    Y[c * no + q] = (float)log10(fmax(out[c * no + q] / pa, 1e-20));
}

// per-column mean and standard deviation (floored) of a float [n][m] matrix
__global__ void k_colstats(const float* __restrict__ A, int64_t n, int m, float* __restrict__ mu,
                           float* __restrict__ sd) {
  const int col = blockIdx.x;
  __shared__ double r1[256], r2[256];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += A[r * m + col];
  r1[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) r1[threadIdx.x] += r1[threadIdx.x + k];
    __syncthreads();
  }
  const double mean = r1[0] / (double)n;
  double v = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double d = A[r * m + col] - mean;
    v += d * d;
  }
  r2[threadIdx.x] = v;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) r2[threadIdx.x] += r2[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mu[col] = (float)mean;
    sd[col] = (float)fmax(sqrt(r2[0] / (double)n), 1e-3);
  }
}

// standardise in place and record the standardised range per column
__global__ void k_standardise(float* __restrict__ A, int64_t n, int m, const float* __restrict__ mu,
                              const float* __restrict__ sd, float* __restrict__ lo, float* __restrict__ hi) {
  const int col = blockIdx.x;
  __shared__ float rlo[256], rhi[256];
  float a = 3e38f, b = -3e38f;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const float x = (A[r * m + col] - mu[col]) / sd[col];
    A[r * m + col] = x;
    a = fminf(a, x);
    b = fmaxf(b, x);
  }
  rlo[threadIdx.x] = a;
  rhi[threadIdx.x] = b;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      rlo[threadIdx.x] = fminf(rlo[threadIdx.x], rlo[threadIdx.x + k]);
      rhi[threadIdx.x] = fmaxf(rhi[threadIdx.x], rhi[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && lo) {
    lo[col] = rlo[0];
    hi[col] = rhi[0];
  }
}

// ---------------------------------------------------------------------------
// Fused persistent inference for networks no wider than 256.  A tile of 64
// cells goes through features, three layers and outputs without leaving the
// chip: two LDS buffers of [64][264] bfloat16 take turns as layer input and
// output.  Eight waves per workgroup, two workgroups per CU: wave w computes
// columns 32 w .. 32 w + 31 of every layer for all 64 cells (4 x 2 blocks of
// v_mfma_f32_16x16x32_bf16), A fragments from LDS, B fragments streamed from
// the zero-padded [256][256] matrices (L2 resident) four K-steps ahead of
// their use.  One workgroup's field loads and epilogues overlap the other's
// products.
constexpr int kFW = 256;         // packed width
constexpr int kFP = kFW + 8;     // LDS row stride in bf16 (16-byte rows, banks spread)
constexpr int kTT = 64;          // cells per tile
constexpr int kTW = 8;           // waves per workgroup
constexpr int kKS = kFW / 32;    // K-steps per layer (inputs zero-padded to 256)
constexpr int kBR = 4;           // B fragments in flight (K-steps ahead)
constexpr int kTR = kTT / kTW;   // field rows per wave

size_t tile_lds(int nl) {
  (void)nl;
  return sizeof(uint16_t) * 2 * kTT * kFP + sizeof(double) * (kTT + kFW) + sizeof(float) * 9 * kFW + sizeof(int) * kTT;
}

// zero-padded [256][256] bf16 copies of W1, W2, W3 (row = output unit)
__global__ void k_pack(const uint16_t* __restrict__ W1, const uint16_t* __restrict__ W2,
                       const uint16_t* __restrict__ W3, int ni, int nh, int no, uint16_t* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 3 * kFW * kFW) return;
  const int which = q / (kFW * kFW), n = (q / kFW) % kFW, k = q % kFW;
  const uint16_t* W = which == 0 ? W1 : (which == 1 ? W2 : W3);
  const int R = which == 2 ? no : nh, K = which == 0 ? ni : nh;
  out[q] = (n < R && k < K) ? W[n * K + k] : (uint16_t)0;
}

struct InferP {
  const float* J;
  int64_t n;
  int nl, ni, nh, no;
  const double* cabs;
  const double* dnu;
  const float *x_mu, *x_sd, *x_lo, *x_hi, *y_mu, *y_sd, *b1, *b2, *b3;
  const uint16_t* Wp;              // [3][256][256]
  float margin, tol;
  double* out;
  uint8_t* ood;
  double* pabs;
};

// acc[mb][cb] = act[16 mb .. + 15][:] W[32 w + 16 cb .. + 15][:]^T.  Lane l
// holds A row l & 15 and B column l & 15 at k = 32 s + 8 (l >> 4) .. + 7;
// accumulator element i is row 4 (l >> 4) + i, column l & 15 of its block.
__device__ __forceinline__ void tile_layer(const uint16_t* act, const uint16_t* __restrict__ W,
                                           f32x4 (&acc)[4][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint16_t* arow = act + (lane & 15) * kFP + 8 * (lane >> 4);
  // opaque per call: the fragment addresses are formed where they are used
  // rather than hoisted out of the tile loop (48 addresses would not fit)
  int wofs = (wave * 32 + (lane & 15)) * kFW + 8 * (lane >> 4);
  asm volatile("" : "+v"(wofs));
  const uint16_t* wrow = W + wofs;
  u16x8 b[kBR][2];
#pragma unroll
  for (int s = 0; s < kBR; ++s)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) b[s][cb] = *reinterpret_cast<const u16x8*>(wrow + cb * 16 * kFW + 32 * s);
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[mb][cb] = f32x4{};
#pragma unroll
  for (int k = 0; k < kKS; ++k) {
    u16x8 a[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) a[mb] = *reinterpret_cast<const u16x8*>(arow + 16 * mb * kFP + 32 * k);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        acc[mb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[mb]),
                                                              __builtin_bit_cast(bf16x8, b[k % kBR][cb]),
                                                              acc[mb][cb], 0, 0, 0);
    if (k + kBR < kKS) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        b[k % kBR][cb] = *reinterpret_cast<const u16x8*>(wrow + cb * 16 * kFW + 32 * (k + kBR));
    }
  }
}

// bfloat16 rounded to nearest even by the conversion instruction (as f2bf)
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// hidden-layer epilogue: bias, SiLU (hardware reciprocal), bfloat16 into the
// other buffer.  Columns past the layer's width have zero weights and zero
// bias, so their activation is SiLU(0) = 0.
__device__ __forceinline__ void tile_hidden(const f32x4 (&acc)[4][2], const float* bias, uint16_t* dst) {
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int col = wave * 32 + 16 * cb + (lane & 15);
    const float b = bias[col];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[mb][cb][i] + b;
        const float h = z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
        dst[(16 * mb + 4 * (lane >> 4) + i) * kFP + col] = bf16_rne(h);
      }
  }
}

// Sums over the wave's 64 lanes of 8 per-lane values v[r] (r = 0..7), by
// halving: at each exchange a lane keeps the half of its values selected by
// one bit of its index and sends the other half.  Returns, on lane L, the
// total of value r = (L >> 3) & 7.
__device__ __forceinline__ double wave_sum8(const double (&v)[8], int lane) {
  const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1;
  double w[4], u[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (b5 ? v[4 + k] : v[k]) + __shfl_xor(b5 ? v[k] : v[4 + k], 32);
#pragma unroll
  for (int k = 0; k < 2; ++k) u[k] = (b4 ? w[2 + k] : w[k]) + __shfl_xor(b4 ? w[k] : w[2 + k], 16);
  double x = (b3 ? u[1] : u[0]) + __shfl_xor(b3 ? u[0] : u[1], 8);
  x += __shfl_xor(x, 4);
  x += __shfl_xor(x, 2);
  x += __shfl_xor(x, 1);
  return x;
}

// Sums over the 16 lanes of each quarter-wave of 16 per-lane values v[s].
// Returns, on lane L, the total of value s = L & 15 over its quarter.
__device__ __forceinline__ double quarter_sum16(const double (&v)[16], int lane) {
  const bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
  double w[8], u[4], t[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = (b3 ? v[8 + k] : v[k]) + __shfl_xor(b3 ? v[k] : v[8 + k], 8);
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = (b2 ? w[4 + k] : w[k]) + __shfl_xor(b2 ? w[k] : w[4 + k], 4);
#pragma unroll
  for (int k = 0; k < 2; ++k) t[k] = (b1 ? u[2 + k] : u[k]) + __shfl_xor(b1 ? u[k] : u[2 + k], 2);
  return (b0 ? t[1] : t[0]) + __shfl_xor(b0 ? t[0] : t[1], 1);
}

__device__ __forceinline__ double bcast_f64(double x, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, src), hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Raw buffer access to one tile's rows: offsets at or past the byte count
// read zero and drop writes (the hardware's range check), so rows past the
// end of the arrays and masked columns need no branches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr uint32_t kOffOut = 0x40000000u;     // an offset past every tile's range

// four waves per SIMD: two workgroups per CU
__global__ void __launch_bounds__(kTW * 64, 4) k_mlp_infer(const InferP p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char tsm[];
  uint16_t* bufA = reinterpret_cast<uint16_t*>(tsm);                // [64][kFP]
  uint16_t* bufB = bufA + kTT * kFP;                                 // [64][kFP]
  double* sPabs = reinterpret_cast<double*>(bufB + kTT * kFP);       // [64]
  double* sW = sPabs + kTT;                                          // [256] cabs dnu (zero past n_lambda)
  float* sMu = reinterpret_cast<float*>(sW + kFW);                   // [256] per input: x_mu, 1 / x_sd,
  float* sRs = sMu + kFW;                                            //   x_lo - margin, x_hi + margin
  float* sLo = sRs + kFW;
  float* sHi = sLo + kFW;
  float* sB1 = sHi + kFW;                                            // [256] per unit: b1, b2, b3, y_mu, y_sd
  float* sB2 = sB1 + kFW;
  float* sB3 = sB2 + kFW;
  float* sYm = sB3 + kFW;
  float* sYs = sYm + kFW;
  int* sBad = reinterpret_cast<int*>(sYs + kFW);                     // [64]
  double* sRow = reinterpret_cast<double*>(bufB);                    // [8][64] row sums (bufB is free then)
  const int nl = p.nl, ni = p.ni, nh = p.nh, no = p.no;

  for (int j = threadIdx.x; j < kFW; j += kTW * 64) {
    sW[j] = j < nl ? p.cabs[j] * p.dnu[j] : 0.0;
    const bool in = j < ni;
    sMu[j] = in ? p.x_mu[j] : 0.0f;
    sRs[j] = in ? 1.0f / p.x_sd[j] : 1.0f;
    sLo[j] = in ? p.x_lo[j] - p.margin : 0.0f;
    sHi[j] = in ? p.x_hi[j] + p.margin : 0.0f;
    sB1[j] = j < nh ? p.b1[j] : 0.0f;
    sB2[j] = j < nh ? p.b2[j] : 0.0f;
    sB3[j] = j < no ? p.b3[j] : 0.0f;
    sYm[j] = j < no ? p.y_mu[j] : 0.0f;
    sYs[j] = j < no ? p.y_sd[j] : 0.0f;
  }
  __syncthreads();

  const int64_t n_tiles = (p.n + kTT - 1) / kTT;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t c0 = t * kTT;
    // the thread index is opaque to the compiler each tile, so that per-row
    // and per-bin addresses and constants are formed (or read from LDS) where
    // they are used instead of being kept in registers across the tile loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int fw = tid >> 6, jb = tid & 63;
    const int rows = p.n - c0 < kTT ? (int)(p.n - c0) : kTT;
    // ---- features of the tile's cells (wave w: rows 8 w .. 8 w + 7; bins
    // lane + 64 q, n_lambda <= 255).  One buffer range per row: bins past
    // n_lambda and rows past the end read zero.
    const int fwu = __builtin_amdgcn_readfirstlane(fw);
    float Jv[kTR][4];
#pragma unroll
    for (int rr = 0; rr < kTR; ++rr) {
      const int64_t c = c0 + fwu * kTR + rr;
      const __amdgpu_buffer_rsrc_t jr = tile_rsrc(p.J + c * nl, c < p.n ? 4u * (uint32_t)nl : 0u);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Jv[rr][q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(jr, 4u * jb + 256u * q, 0, 0));
    }
    // absorbed power per cell in FP64: sum over bins of C_abs J dnu; then
    // lane L finishes row 8 w + ((L >> 3) & 7): P_abs, its reciprocal and
    // the last input log10 P_abs (mantissa in FP32 plus exponent)
    double v[kTR];
#pragma unroll
    for (int rr = 0; rr < kTR; ++rr) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) s = fma(sW[jb + 64 * q], (double)Jv[rr][q], s);
      v[rr] = s;
    }
    const double tot = wave_sum8(v, jb);
    const double inv_l = tot > 0.0 ? 1.0 / tot : 0.0;
    const double pa_l = 4.0 * kPi * tot;
    int e2 = 0;
    const float m2 = (float)frexp(fmax(pa_l, 1e-300), &e2);
    const float lpa_l = log10f(m2) + (float)e2 * 0.301029995663981f;
    if ((jb & 7) == 0) sPabs[fw * kTR + (jb >> 3)] = pa_l;
#pragma unroll
    for (int rr = 0; rr < kTR; ++rr) {
      const int row = fw * kTR + rr;
      const double inv = bcast_f64(inv_l, 8 * rr), pa = bcast_f64(pa_l, 8 * rr);
      const float lpa = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(uint32_t, lpa_l), 8 * rr));
      bool bad = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // Every operand is read unconditionally (a read under a condition
        // becomes a branch).  Past the inputs (j >= n_in) the tables hold
        // C_abs dnu = 0, x_mu = 0, 1 / x_sd = 1 and a range [0, 0], so x = 0
        // exactly there, never flagged and multiplied by zero weights; a row
        // past the end has a zero field and finite inputs, and no outputs.
        const int j = jb + 64 * q;
        const double w = sW[j];
        const float mu = sMu[j], rsd = sRs[j], lo = sLo[j], hi = sHi[j];
        const float fj = (float)(w * (double)Jv[rr][q] * inv);
        const float x = ((j == nl ? lpa : fj) - mu) * rsd;
        bad |= (x < lo) | (x > hi);
        bufA[row * kFP + j] = bf16_rne(x);
      }
      // a dark cell (no absorbed power) has the exact answer F = 0 (the
      // molecule stays in its ground state), whatever its inputs look like
      const int flag = __any(bad) && pa > 0.0;
      if (jb == 0) sBad[row] = flag;
    }
    __syncthreads();

    f32x4 acc[4][2];
    tile_layer(bufA, p.Wp, acc);
    tile_hidden(acc, sB1, bufB);
    __syncthreads();
    tile_layer(bufB, p.Wp + kFW * kFW, acc);
    tile_hidden(acc, sB2, bufA);
    __syncthreads();
    tile_layer(bufA, p.Wp + 2 * kFW * kFW, acc);

    // ---- outputs F = 10^(y sd + mu) P_abs and their per-cell sums over this
    // wave's 32 columns.  10^z = 2^(z log2 10) in FP32 (relative error
    // ~1e-6 at |z| ~ 10): the network's own error (BF16 operands, ~1e-3)
    // dwarfs it
    int ot = threadIdx.x;
    asm volatile("" : "+v"(ot));
    const int lane = ot & 63, wave = ot >> 6;
    // z log2 10 = y' a + c with a = sd log2 10, c = (b3 sd + mu) log2 10;
    // a column past the network's width has a = 0, c = -inf (F = 0).  The
    // exponent is capped at 2^127 so that F stays finite and a dark cell's
    // F = 10^z * 0 is exactly zero.
    float ea[2], ec[2];
    uint32_t co[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int col = wave * 32 + 16 * cb + (lane & 15);
      const bool on = col < no;
      ea[cb] = on ? sYs[col] * 3.32192809488736f : 0.0f;
      ec[cb] = on ? fmaf(sB3[col], sYs[col], sYm[col]) * 3.32192809488736f : -__builtin_inff();
      co[cb] = on ? 8u * col : kOffOut;
    }
    const __amdgpu_buffer_rsrc_t orr = tile_rsrc(p.out + c0 * no, (uint32_t)(rows * no) * 8u);
    double rs[16];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * mb + 4 * (lane >> 4) + i;
        const double pa = fmax(sPabs[row], 0.0);
        const uint32_t ro = 8u * (uint32_t)(row * no);
        double F2 = 0.0;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const float e = __builtin_amdgcn_exp2f(fminf(fmaf(acc[mb][cb][i], ea[cb], ec[cb]), 127.0f));
          const double F = (double)e * pa;
          const uint64_t fb = __builtin_bit_cast(uint64_t, F);
          typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
          const u32x2 fv = {(uint32_t)fb, (uint32_t)(fb >> 32)};
          __builtin_amdgcn_raw_buffer_store_b64(fv, orr, ro + co[cb], 0, 0);
          F2 += F;
        }
        rs[4 * mb + i] = F2;
      }
    {
      // lane L: sum over this wave's columns of row 16 (s >> 2) + 4 (L >> 4) + (s & 3), s = L & 15
      const double x = quarter_sum16(rs, lane);
      const int s16 = lane & 15;
      sRow[wave * kTT + 16 * (s16 >> 2) + 4 * (lane >> 4) + (s16 & 3)] = x;
    }
    __syncthreads();
    if (threadIdx.x < kTT && c0 + threadIdx.x < p.n) {
      const int row = threadIdx.x;
      double tot = 0.0;
      for (int w = 0; w < kTW; ++w) tot += sRow[w * kTT + row];
      const double pa = sPabs[row];
      const int bal = !(fabs(tot - pa) <= p.tol * pa);
      p.ood[c0 + row] = (uint8_t)(sBad[row] | (bal << 1));
      p.pabs[c0 + row] = pa;
    }
    // the buffers and row sums are rewritten by the next tile
    __syncthreads();
  }
}

}  // namespace

struct pah_mlp {
  int ni, nh, no, batch;
  int infer_blocks = -1;            // grid of the persistent inference kernel
  MlpLayout L;
  unsigned char* st = nullptr;
  std::string err;
};

namespace {

int32_t mfail(pah_mlp* m, int32_t code, const std::string& s) {
  if (m) m->err = s;
  return code;
}

template <typename T>
T* at(pah_mlp* m, uint64_t off) { return reinterpret_cast<T*>(m->st + off); }

hipError_t refresh_all(pah_mlp* m, hipStream_t s) {
  const MlpLayout& L = m->L;
  float* P = at<float>(m, L.params);
  struct { uint64_t o; int64_t n; uint64_t h; } mats[3] = {
      {L.oW1, (int64_t)m->nh * m->ni, L.W1h}, {L.oW2, (int64_t)m->nh * m->nh, L.W2h},
      {L.oW3, (int64_t)m->no * m->nh, L.W3h}};
  for (auto& w : mats)
    k_refresh<<<(unsigned)((w.n + 255) / 256), 256, 0, s>>>(P + w.o, w.n, at<uint16_t>(m, w.h));
  return hipGetLastError();
}

// forward on bf16 inputs already in X16 (rows n <= batch); Y fp32 standardised
hipError_t forward(pah_mlp* m, int64_t n, const uint16_t* X16, float* Y, hipStream_t s) {
  const MlpLayout& L = m->L;
  const float* P = at<float>(m, L.params);
  GemmP g{};
  g.M = (int)n; g.N = m->nh; g.K = m->ni; g.A = X16; g.lda = m->ni; g.ta = 0;
  g.B = at<uint16_t>(m, L.W1h); g.ldb = m->ni; g.tb = 1; g.bias = P + L.ob1;
  g.C = at<float>(m, L.Z1); g.ldc = m->nh; g.H = at<uint16_t>(m, L.H1); g.ldh = m->nh;
  hipError_t e = gemm<EPI_SILU>(g, s);
  if (e != hipSuccess) return e;
  g.K = m->nh; g.A = at<uint16_t>(m, L.H1); g.lda = m->nh; g.B = at<uint16_t>(m, L.W2h); g.ldb = m->nh;
  g.bias = P + L.ob2; g.C = at<float>(m, L.Z2); g.H = at<uint16_t>(m, L.H2);
  e = gemm<EPI_SILU>(g, s);
  if (e != hipSuccess) return e;
  g.N = m->no; g.A = at<uint16_t>(m, L.H2); g.B = at<uint16_t>(m, L.W3h); g.bias = P + L.ob3;
  g.C = Y; g.ldc = m->no; g.H = nullptr;
  return gemm<EPI_F32>(g, s);
}

// backward from dY16 (bf16, rows n): grads of all parameters into the grads block
hipError_t backward(pah_mlp* m, int64_t n, hipStream_t s) {
  const MlpLayout& L = m->L;
  float* G = at<float>(m, L.grads);
  const int ni = m->ni, nh = m->nh, no = m->no;
  const uint16_t* dY = at<uint16_t>(m, L.dY16);
  GemmP g{};
  // dW3 [no][nh] = dY^T H2
  g.M = no; g.N = nh; g.K = (int)n; g.A = dY; g.lda = no; g.ta = 1;
  g.B = at<uint16_t>(m, L.H2); g.ldb = nh; g.tb = 0; g.C = G + L.oW3; g.ldc = nh;
  hipError_t e = gemm_f32_split(g, at<float>(m, L.part), s);
  k_colsum<<<(no + 63) / 64, 64 * kColRows, 0, s>>>(dY, n, no, G + L.ob3);
  // dZ2 = (dY W3) * silu'(Z2); W3 [no][nh] read as (k=o, n=j) -> W3h with tb = 0
  g = GemmP{};
  g.M = (int)n; g.N = nh; g.K = no; g.A = dY; g.lda = no; g.ta = 0;
  g.B = at<uint16_t>(m, L.W3h); g.ldb = nh; g.tb = 0;
  g.H = at<uint16_t>(m, L.dZ2); g.ldh = nh; g.Z = at<float>(m, L.Z2); g.ldz = nh;
  if (e == hipSuccess) e = gemm<EPI_DSILU>(g, s);
  // dW2 [nh][nh] = dZ2^T H1
  g = GemmP{};
  g.M = nh; g.N = nh; g.K = (int)n; g.A = at<uint16_t>(m, L.dZ2); g.lda = nh; g.ta = 1;
  g.B = at<uint16_t>(m, L.H1); g.ldb = nh; g.tb = 0; g.C = G + L.oW2; g.ldc = nh;
  if (e == hipSuccess) e = gemm_f32_split(g, at<float>(m, L.part), s);
  k_colsum<<<(nh + 63) / 64, 64 * kColRows, 0, s>>>(at<uint16_t>(m, L.dZ2), n, nh, G + L.ob2);
  // dZ1 = (dZ2 W2) * silu'(Z1)
  g = GemmP{};
  g.M = (int)n; g.N = nh; g.K = nh; g.A = at<uint16_t>(m, L.dZ2); g.lda = nh; g.ta = 0;
  g.B = at<uint16_t>(m, L.W2h); g.ldb = nh; g.tb = 0;
  g.H = at<uint16_t>(m, L.dZ1); g.ldh = nh; g.Z = at<float>(m, L.Z1); g.ldz = nh;
  if (e == hipSuccess) e = gemm<EPI_DSILU>(g, s);
  // dW1 [nh][ni] = dZ1^T X
  g = GemmP{};
  g.M = nh; g.N = ni; g.K = (int)n; g.A = at<uint16_t>(m, L.dZ1); g.lda = nh; g.ta = 1;
  g.B = at<uint16_t>(m, L.X16); g.ldb = ni; g.tb = 0; g.C = G + L.oW1; g.ldc = ni;
  if (e == hipSuccess) e = gemm_f32_split(g, at<float>(m, L.part), s);
  k_colsum<<<(nh + 63) / 64, 64 * kColRows, 0, s>>>(at<uint16_t>(m, L.dZ1), n, nh, G + L.ob1);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

extern "C" {

int32_t pah_mlp_state_bytes(int32_t n_in, int32_t n_h, int32_t n_out, int32_t batch, uint64_t* bytes) {
  if (n_in < 1 || n_h < 1 || n_out < 1 || batch < 1 || !bytes || n_in > 8192 || n_h > 8192 || n_out > 8192)
    return MCRT_E_INVALID;
  *bytes = mlp_layout(n_in, n_h, n_out, batch).total;
  return MCRT_OK;
}

int32_t pah_mlp_create(int32_t n_in, int32_t n_h, int32_t n_out, int32_t batch, void* state,
                       uint64_t state_bytes, pah_mlp** out) {
  if (!out) return MCRT_E_INVALID;
  *out = nullptr;
  uint64_t need = 0;
  if (pah_mlp_state_bytes(n_in, n_h, n_out, batch, &need) != MCRT_OK || !state) return MCRT_E_INVALID;
  if (state_bytes < need) return MCRT_E_CAPACITY;
  pah_mlp* m = new (std::nothrow) pah_mlp();
  if (!m) return MCRT_E_INVALID;
  m->ni = n_in; m->nh = n_h; m->no = n_out; m->batch = batch;
  m->L = mlp_layout(n_in, n_h, n_out, batch);
  m->st = static_cast<unsigned char*>(state);
  *out = m;
  return MCRT_OK;
}

void pah_mlp_destroy(pah_mlp* m) { delete m; }

const char* pah_mlp_last_error(const pah_mlp* m) { return m ? m->err.c_str() : "null network"; }

int32_t pah_mlp_offsets(const pah_mlp* m, uint64_t* off, int32_t n_off) {
  if (!m || !off || n_off < 32) return MCRT_E_INVALID;
  const MlpLayout& L = m->L;
  const uint64_t v[32] = {L.params, L.grads, L.adam_m, L.adam_v, L.n_params, L.oW1, L.ob1, L.oW2,
                          L.ob2, L.oW3, L.ob3, L.W1h, L.W2h, L.W3h, L.x_mu, L.x_sd, L.x_lo, L.x_hi,
                          L.y_mu, L.y_sd, L.X16, L.Z1, L.H1, L.Z2, L.H2, L.Y, L.dY16, L.dZ2, L.dZ1,
                          L.loss, L.Wpk, L.total};
  std::memcpy(off, v, sizeof v);
  return MCRT_OK;
}

int32_t pah_mlp_load(pah_mlp* m, const float* params, hipStream_t s) {
  if (!m || !params) return MCRT_E_INVALID;
  const MlpLayout& L = m->L;
  hipError_t e = hipMemcpyAsync(m->st + L.params, params, 4 * L.n_params, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(m->st + L.adam_m, 0, 4 * L.n_params, s);
  if (e == hipSuccess) e = hipMemsetAsync(m->st + L.adam_v, 0, 4 * L.n_params, s);
  if (e == hipSuccess) e = refresh_all(m, s);
  if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_mlp_set_norm(pah_mlp* m, const float* x_mu, const float* x_sd, const float* x_lo,
                         const float* x_hi, const float* y_mu, const float* y_sd, hipStream_t s) {
  if (!m || !x_mu || !x_sd || !x_lo || !x_hi || !y_mu || !y_sd) return MCRT_E_INVALID;
  const MlpLayout& L = m->L;
  const float* src[6] = {x_mu, x_sd, x_lo, x_hi, y_mu, y_sd};
  const uint64_t dst[6] = {L.x_mu, L.x_sd, L.x_lo, L.x_hi, L.y_mu, L.y_sd};
  for (int k = 0; k < 6; ++k) {
    const uint64_t n = k < 4 ? (uint64_t)m->ni : (uint64_t)m->no;
    const hipError_t e = hipMemcpyAsync(m->st + dst[k], src[k], 4 * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  }
  return MCRT_OK;
}

int32_t pah_mlp_forward(pah_mlp* m, const float* X, int32_t n, float* Y, hipStream_t s) {
  if (!m || !X || !Y) return MCRT_E_INVALID;
  if (n < 1 || n > m->batch) return mfail(m, MCRT_E_CAPACITY, "n outside 1..batch");
  const int64_t nx = (int64_t)n * m->ni;
  k_to_bf16<<<(unsigned)((nx + 255) / 256), 256, 0, s>>>(X, nx, at<uint16_t>(m, m->L.X16));
  const hipError_t e = forward(m, n, at<uint16_t>(m, m->L.X16), Y, s);
  if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_mlp_train_step(pah_mlp* m, const float* X, const float* T, int32_t n, float lr,
                           int32_t step, hipStream_t s) {
  if (!m || !X || !T) return MCRT_E_INVALID;
  if (n < 1 || n > m->batch) return mfail(m, MCRT_E_CAPACITY, "n outside 1..batch");
  if (step < 1) return mfail(m, MCRT_E_INVALID, "step counts from 1");
  const MlpLayout& L = m->L;
  const int64_t nx = (int64_t)n * m->ni;
  k_to_bf16<<<(unsigned)((nx + 255) / 256), 256, 0, s>>>(X, nx, at<uint16_t>(m, L.X16));
  hipError_t e = forward(m, n, at<uint16_t>(m, L.X16), at<float>(m, L.Y), s);
  if (e == hipSuccess) e = hipMemsetAsync(m->st + L.loss, 0, 4, s);
  if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  k_loss<<<256, 256, 0, s>>>(at<float>(m, L.Y), T, n, m->no, at<uint16_t>(m, L.dY16), at<float>(m, L.loss));
  e = backward(m, n, s);
  if (e == hipSuccess && lr != 0.0f) {
    const double b1 = 0.9, b2 = 0.999;
    const int64_t np = (int64_t)L.n_params;
    k_adam<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(
        at<float>(m, L.params), at<float>(m, L.grads), at<float>(m, L.adam_m), at<float>(m, L.adam_v),
        np, lr, (float)b1, (float)b2, 1e-8f, (float)(1.0 - pow(b1, step)), (float)(1.0 - pow(b2, step)));
    e = refresh_all(m, s);
  }
  if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_mlp_prepare(pah_mlp* m, const pah_ctx* ctx, const float* J, const double* out,
                        const double* pabs, int64_t n, float* X, float* Y, hipStream_t s) {
  if (!m || !ctx || !J || !out || !pabs || !X || !Y || n < 2) return MCRT_E_INVALID;
  const pah_desc& d = pah_ctx_desc(ctx);
  if (d.n_lambda + 1 != m->ni || d.n_bands + d.n_lambda != m->no)
    return mfail(m, MCRT_E_INVALID, "network shape does not match the PAH model");
  const double* dnu = pah_ctx_dnu(ctx);
  if (!dnu) return mfail(m, MCRT_E_STATE, "PAH tables not built");
  const MlpLayout& L = m->L;
  k_prep<<<(unsigned)n, 256, 0, s>>>(J, out, pabs, n, d.n_lambda, m->no, d.cabs, dnu, X, Y);
  k_colstats<<<m->ni, 256, 0, s>>>(X, n, m->ni, at<float>(m, L.x_mu), at<float>(m, L.x_sd));
  k_colstats<<<m->no, 256, 0, s>>>(Y, n, m->no, at<float>(m, L.y_mu), at<float>(m, L.y_sd));
  k_standardise<<<m->ni, 256, 0, s>>>(X, n, m->ni, at<float>(m, L.x_mu), at<float>(m, L.x_sd),
                                      at<float>(m, L.x_lo), at<float>(m, L.x_hi));
  k_standardise<<<m->no, 256, 0, s>>>(Y, n, m->no, at<float>(m, L.y_mu), at<float>(m, L.y_sd),
                                      nullptr, nullptr);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  return MCRT_OK;
}

int32_t pah_surrogate_infer(pah_mlp* m, const pah_ctx* ctx, const float* J, int64_t n, double* out,
                            uint8_t* ood, double* pabs, float in_margin, float balance_tol,
                            hipStream_t s) {
  if (!m || !ctx || !J || !out || !ood || !pabs) return MCRT_E_INVALID;
  if (n < 0) return mfail(m, MCRT_E_INVALID, "n < 0");
  const pah_desc& d = pah_ctx_desc(ctx);
  if (d.n_lambda + 1 != m->ni || d.n_bands + d.n_lambda != m->no)
    return mfail(m, MCRT_E_INVALID, "network shape does not match the PAH model");
  const double* dnu = pah_ctx_dnu(ctx);
  if (!dnu) return mfail(m, MCRT_E_STATE, "PAH tables not built");
  const MlpLayout& L = m->L;
  if (n == 0) return MCRT_OK;
  if (m->ni <= kFW && m->nh <= kFW && m->no <= kFW) {
    k_pack<<<(3 * kFW * kFW + 255) / 256, 256, 0, s>>>(at<uint16_t>(m, L.W1h), at<uint16_t>(m, L.W2h),
                                                        at<uint16_t>(m, L.W3h), m->ni, m->nh, m->no,
                                                        at<uint16_t>(m, L.Wpk));
    InferP p{};
    p.J = J; p.n = n; p.nl = d.n_lambda; p.ni = m->ni; p.nh = m->nh; p.no = m->no;
    p.cabs = d.cabs; p.dnu = dnu;
    p.x_mu = at<float>(m, L.x_mu); p.x_sd = at<float>(m, L.x_sd);
    p.x_lo = at<float>(m, L.x_lo); p.x_hi = at<float>(m, L.x_hi);
    p.y_mu = at<float>(m, L.y_mu); p.y_sd = at<float>(m, L.y_sd);
    const float* P = at<float>(m, L.params);
    p.b1 = P + L.ob1; p.b2 = P + L.ob2; p.b3 = P + L.ob3;
    p.Wp = at<uint16_t>(m, L.Wpk);
    p.margin = in_margin; p.tol = balance_tol;
    p.out = out; p.ood = ood; p.pabs = pabs;
    if (m->infer_blocks < 0) {
      int dev = 0, ncu = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_infer, kTW * 64, tile_lds(d.n_lambda)) !=
              hipSuccess || per_cu < 1)
        per_cu = 1;
      m->infer_blocks = ncu * per_cu;
    }
    const int64_t tiles = (n + kTT - 1) / kTT;
    const int64_t blocks = tiles < m->infer_blocks ? tiles : m->infer_blocks;
    k_mlp_infer<<<(unsigned)blocks, kTW * 64, tile_lds(d.n_lambda), s>>>(p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
    return MCRT_OK;
  }
  for (int64_t c0 = 0; c0 < n; c0 += m->batch) {
    const int64_t nc = n - c0 < m->batch ? n - c0 : m->batch;
    k_mlp_in<<<(unsigned)nc, 256, sizeof(float) * m->ni, s>>>(J + c0 * d.n_lambda, nc, d.n_lambda, d.cabs, dnu, at<float>(m, L.x_mu),
                                           at<float>(m, L.x_sd), at<float>(m, L.x_lo), at<float>(m, L.x_hi),
                                           in_margin, at<uint16_t>(m, L.X16), pabs + c0, ood + c0);
    hipError_t e = forward(m, nc, at<uint16_t>(m, L.X16), at<float>(m, L.Y), s);
    if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
    k_mlp_out<<<(unsigned)nc, 256, 0, s>>>(at<float>(m, L.Y), nc, m->no, at<float>(m, L.y_mu),
                                            at<float>(m, L.y_sd), pabs + c0, balance_tol, out + c0 * m->no,
                                            ood + c0);
    e = hipGetLastError();
    if (e != hipSuccess) return mfail(m, MCRT_E_HIP, hipGetErrorString(e));
  }
  return MCRT_OK;
}

}  // extern "C"
