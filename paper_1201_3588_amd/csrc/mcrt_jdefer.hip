// Deferred path-length tally (the mean-intensity estimator of Lucy 1999 that
// the paper's method accumulates per cell and wavelength).  Random 64-bit
// atomics into the tally are limited by the L2 atomic units whatever the
// table size, so the transport instead appends one record per path segment,
// (tally index << 24) | fixed-point length, contiguously per wave.  Here the
// records are added to the tally with streaming passes and LDS sums:
//   count    histogram of records per (bucket, tile)
//   scan     exclusive scan of the counts, bucket-major: each bucket's records
//            become one contiguous range, ordered by tile
//   scatter  records to their bucket ranges (sub-tiles sorted in LDS first)
//   items    work items of at most kPart records per bucket
//   sum      per item, u32 partial sums of its bucket (kBucketSlots tally
//            words) in LDS (a carry past 2^32 goes straight to the tally),
//            then one add per tally word: plain for a bucket of one item,
//            atomic for a bucket shared by several items.
// A tally of many buckets is partitioned in two levels, so that every
// scatter writes long runs: first into coarse ranges of fpc buckets, then
// each coarse range, tile by tile, into its buckets.
// Integer sums do not depend on order, so the tally equals the one the
// atomic path gives, bit for bit.
#include "mcrt_internal.h"

namespace mcrt {

namespace {

constexpr int kScanBlocks = 256;
constexpr uint64_t kPart = 1ull << 20;      // records per summing work item
constexpr int kLoads = 16;                  // record loads per thread in flight (count, sum)
constexpr unsigned long long kValMask = (1ull << kRecValBits) - 1ull;

// Unsigned 32-bit division by an invariant divisor as a multiply-high, two
// shifts and an add (Granlund & Montgomery, "Division by invariant integers
// using multiplication", PLDI 1994, Sec. 4): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1 (< 2^32), t = mulhi(m, n) gives
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) exactly for every
// 32-bit n.  The emulated division it replaces costs about twenty VALU
// instructions per record.
struct UDiv {
  uint32_t d, m, s1, s2;
};

UDiv make_udiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return UDiv{d, (uint32_t)m, l < 1 ? l : 1u, l > 0 ? l - 1 : 0u};
}

__device__ __forceinline__ uint32_t udiv(uint32_t n, const UDiv& D) {
  const uint32_t t = __umulhi(D.m, n);
  return (t + ((n - t) >> D.s1)) >> D.s2;
}

// bucket of a record among nb buckets of D.d tally words from slot0
__device__ __forceinline__ uint32_t bucket_of(unsigned long long r, uint64_t slot0, const UDiv& D, uint32_t nb) {
  const uint64_t slot = r >> kRecValBits;
  const uint64_t d = slot >= slot0 ? slot - slot0 : 0;
  // 32-bit division when the offset fits (every tally below 2^32 words)
  const uint64_t b = d < (1ull << 32) ? (uint64_t)udiv((uint32_t)d, D) : d / D.d;
  return b < nb ? (uint32_t)b : nb - 1;
}

// Where the buckets' records are after the last partition pass.  One level:
// bucket b starts at offs[b nt].  Two levels: bucket b = c fpc + f starts at
// entry (c, f, 0) of the level-2 counts, laid out [c][f][tile of c] with
// tb[c] tiles before coarse range c.
struct BucketMap {
  const uint64_t* offs;
  const uint32_t* tb;       // null for one level
  uint64_t nt;
  uint32_t fpc, nc, nb;     // nb: buckets
};

__device__ __forceinline__ uint64_t bucket_start(const BucketMap& M, uint32_t b, uint64_t n) {
  if (b >= M.nb) return n;
  if (!M.tb) return M.offs[(uint64_t)b * M.nt];
  const uint32_t c = b / M.fpc, f = b - c * M.fpc;
  const uint32_t t0 = M.tb[c], ntc = M.tb[c + 1] - t0;
  const uint64_t idx = (uint64_t)t0 * M.fpc + (uint64_t)f * ntc;
  return idx < (uint64_t)M.tb[M.nc] * M.fpc ? M.offs[idx] : n;
}

// level-2 tile g: its coarse range c (largest c with tb[c] <= g) and index k
__device__ __forceinline__ bool tile2(const uint32_t* tb, uint32_t nc, uint32_t g, uint32_t& c, uint32_t& k) {
  if (g >= tb[nc]) return false;
  uint32_t lo = 0, hi = nc;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tb[mid] <= g) lo = mid; else hi = mid;
  }
  c = lo;
  k = g - tb[lo];
  return true;
}

// Blocks are dealt to the chip's 8 XCDs round-robin (block b to XCD b mod 8).
// The tile of block b among `used` tiles, chosen so that each XCD takes one
// contiguous range of tiles: the runs of a bucket in neighbouring tiles meet
// in one cache line, which is then completed in one L2 instead of two (the
// same holds for neighbouring words of the per-tile counts).  The grid needs
// at least 8 ceil(used / 8) blocks; false for a block without a tile.
constexpr uint64_t kXcds = 8;

__device__ __forceinline__ bool xcd_tile(uint64_t b, uint64_t used, uint64_t& t) {
  const uint64_t q = (used + kXcds - 1) / kXcds;
  const uint64_t i = b / kXcds;
  if (i >= q) return false;
  t = (b % kXcds) * q + i;
  return t < used;
}

__device__ __forceinline__ uint64_t n_records(const unsigned long long* hdr, uint64_t cap) {
  const uint64_t n = hdr[0];
  return n < cap ? n : cap;
}

// histogram of the records [a, e) over nb buckets of D.d words from slot0
__device__ __forceinline__ void count_range(const unsigned long long* __restrict__ rec, uint64_t a, uint64_t e,
                                            uint64_t slot0, const UDiv& D, uint32_t nb, uint32_t* h) {
  // kLoads records per thread in flight: the passes over the records are
  // bound by the bytes a CU keeps in flight
  for (uint64_t k = a + threadIdx.x; k < e; k += kLoads * 256) {
    unsigned long long r[kLoads];
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const uint64_t kk = k + (uint64_t)q * 256;
      r[q] = kk < e ? rec[kk] : ~0ull;
    }
#pragma unroll
    for (int q = 0; q < kLoads; ++q)
      if (r[q] != ~0ull) atomicAdd(&h[bucket_of(r[q], slot0, D, nb)], 1u);
  }
}

// level 1: tile t of the record array; counts [bucket][tile]
__global__ void __launch_bounds__(256) k_jr_count(const unsigned long long* __restrict__ rec,
                                                 const unsigned long long* hdr, uint64_t cap, uint32_t nb,
                                                 UDiv span, uint64_t nt, uint64_t* __restrict__ counts) {
  extern __shared__ uint32_t h[];
  const uint64_t n = n_records(hdr, cap);
  const uint64_t used = (n + kTile1 - 1) / kTile1;
  uint64_t t;
  if (xcd_tile(blockIdx.x, used, t)) {
    for (uint32_t i = threadIdx.x; i < nb; i += 256) h[i] = 0u;
    __syncthreads();
    const uint64_t a = t * kTile1, e = a + kTile1 < n ? a + kTile1 : n;
    count_range(rec, a, e, 0, span, nb, h);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += 256) counts[(uint64_t)i * nt + t] = h[i];
  }
  // the tiles past the last record: block t writes their zero counts
  if (blockIdx.x >= used && blockIdx.x < nt)
    for (uint32_t i = threadIdx.x; i < nb; i += 256) counts[(uint64_t)i * nt + blockIdx.x] = 0ull;
}

// tiles of each coarse range for level 2: tb[c] = tiles before range c
// (ranges from the level-1 offsets), tb[nc] = all tiles
__global__ void __launch_bounds__(1024) k_jr_dir(const uint64_t* __restrict__ offs1, const unsigned long long* hdr,
                                                uint64_t cap, uint32_t nc, uint64_t nt, uint32_t* __restrict__ tb) {
  __shared__ uint32_t s[1024];
  const uint64_t n = n_records(hdr, cap);
  const uint32_t per = (nc + 1023) / 1024, c0 = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t c = c0; c < c0 + per && c < nc; ++c) {
    const uint64_t lo = offs1[(uint64_t)c * nt], hi = c + 1 < nc ? offs1[(uint64_t)(c + 1) * nt] : n;
    loc += (uint32_t)((hi - lo + kTile1 - 1) / kTile1);
  }
  s[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - loc;
  for (uint32_t c = c0; c < c0 + per && c < nc; ++c) {
    tb[c] = run;
    const uint64_t lo = offs1[(uint64_t)c * nt], hi = c + 1 < nc ? offs1[(uint64_t)(c + 1) * nt] : n;
    run += (uint32_t)((hi - lo + kTile1 - 1) / kTile1);
  }
  if (threadIdx.x == 1023) tb[nc] = s[1023];
}

// level 2: tile g is tile k of coarse range c; counts at [c][f][k]
__global__ void __launch_bounds__(256) k_jr_count2(const unsigned long long* __restrict__ rec,
                                                  const unsigned long long* hdr, uint64_t cap, uint32_t fpc,
                                                  uint32_t nc, uint64_t nt, const uint64_t* __restrict__ offs1,
                                                  const uint32_t* __restrict__ tb, UDiv span,
                                                  uint64_t* __restrict__ counts2) {
  extern __shared__ uint32_t h[];
  uint64_t g;
  uint32_t c, k;
  if (!xcd_tile(blockIdx.x, tb[nc], g) || !tile2(tb, nc, (uint32_t)g, c, k)) return;
  const uint64_t n = n_records(hdr, cap);
  const uint64_t lo = offs1[(uint64_t)c * nt], hi = c + 1 < nc ? offs1[(uint64_t)(c + 1) * nt] : n;
  for (uint32_t i = threadIdx.x; i < fpc; i += 256) h[i] = 0u;
  __syncthreads();
  const uint64_t a = lo + (uint64_t)k * kTile1, e = a + kTile1 < hi ? a + kTile1 : hi;
  count_range(rec, a, e, (uint64_t)c * fpc * kBucketSlots, span, fpc, h);
  __syncthreads();
  const uint32_t t0 = tb[c], ntc = tb[c + 1] - t0;
  for (uint32_t f = threadIdx.x; f < fpc; f += 256)
    counts2[(uint64_t)t0 * fpc + (uint64_t)f * ntc + k] = h[f];
}

// exclusive scan of v[0, n) in place: block sums, their scan, then each block
// rescans its range from its base
__global__ void __launch_bounds__(256) k_scan_sums(const uint64_t* __restrict__ v, uint64_t n,
                                                  unsigned long long* __restrict__ bsum) {
  __shared__ unsigned long long s[256];
  const uint64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
  const uint64_t a = blockIdx.x * chunk, e = a + chunk < n ? a + chunk : n;
  unsigned long long acc = 0;
  for (uint64_t k = a + threadIdx.x; k < e; k += 256) acc += v[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ void k_scan_top(unsigned long long* bsum) {
  if (threadIdx.x != 0) return;
  unsigned long long run = 0;
  for (int g = 0; g < kScanBlocks; ++g) {
    const unsigned long long x = bsum[g];
    bsum[g] = run;
    run += x;
  }
  bsum[kScanBlocks] = run;
}

__global__ void __launch_bounds__(256) k_scan_apply(uint64_t* __restrict__ v, uint64_t n,
                                                   const unsigned long long* __restrict__ bsum) {
  __shared__ uint64_t s[256];
  const uint64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
  const uint64_t a = blockIdx.x * chunk, e = a + chunk < n ? a + chunk : n;
  uint64_t carry = bsum[blockIdx.x];
  for (uint64_t k0 = a; k0 < e; k0 += 256) {
    const uint64_t k = k0 + threadIdx.x;
    const uint64_t x = k < e ? v[k] : 0ull;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {      // inclusive scan (Hillis-Steele)
      const uint64_t y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0ull;
      __syncthreads();
      s[threadIdx.x] += y;
      __syncthreads();
    }
    if (k < e) v[k] = carry + s[threadIdx.x] - x;
    const uint64_t tot = s[255];
    __syncthreads();
    carry += tot;
  }
}

// Block-wide exclusive scan of v[0, n) in LDS with NT threads; returns the
// total.  Each thread sums its run of entries, the runs are scanned within
// each wave by shuffles and across the NT / 64 waves through part (LDS
// scratch of NT / 64 words): two barriers in all.
template <int NT>
__device__ uint32_t block_exclusive_scan(uint32_t* v, uint32_t n, uint32_t* part) {
  const uint32_t per = (n + NT - 1) / NT, a = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t i = a; i < a + per && i < n; ++i) loc += v[i];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint32_t inc = loc;                                  // inclusive within the wave
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63u) part[wave] = inc;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < NT / 64; ++w) {
    const uint32_t t = part[w];
    before += w < wave ? t : 0u;
    total += t;
  }
  uint32_t run = before + inc - loc;
  for (uint32_t i = a; i < a + per && i < n; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

// The records [a, e) of src, sub-tile by sub-tile sorted by bucket in LDS
// and written as contiguous runs (consecutive threads, consecutive
// addresses) from run[b], the next free position of bucket b in dst.
template <int NT>
__device__ void scatter_range(const unsigned long long* __restrict__ src, uint64_t a, uint64_t e, uint64_t slot0,
                              const UDiv& span, uint32_t nb, uint64_t* run, uint32_t* pre, unsigned long long* srt,
                              uint32_t* part, unsigned long long* __restrict__ dst, uint64_t n, uint32_t sub) {
  constexpr int kMaxPer = 16;                                         // sub <= 16 NT
  for (uint64_t s0 = a; s0 < e; s0 += sub) {
    const uint32_t m = (uint32_t)(e - s0 < sub ? e - s0 : sub);
    unsigned long long r[kMaxPer];
    uint32_t bk[kMaxPer], rk[kMaxPer];
    // all loads first (positions past m re-read record s0 and are dropped),
    // so that a wave has its whole share in flight at once
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      r[q] = src[s0 + (k < m ? k : 0u)];
    }
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      bk[q] = bucket_of(r[q], slot0, span, nb);
      if (k < m) rk[q] = atomicAdd(&pre[bk[q]], 1u);
    }
    __syncthreads();
    block_exclusive_scan<NT>(pre, nb, part);
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      if (k < m) srt[pre[bk[q]] + rk[q]] = r[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      const uint32_t kk = k < m ? k : 0u;
      const unsigned long long x = srt[kk];
      const uint32_t b = bucket_of(x, slot0, span, nb);
      const uint64_t d = run[b] + (kk - pre[b]);
      // plain store: a bucket's runs are completed across sub-tiles in the L2
      // (non-temporal stores made this pass 23 % slower)
      if (k < m && d < n) dst[d] = x;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += NT) {
      const uint32_t next = i + 1 < nb ? pre[i + 1] : m;
      run[i] += next - pre[i];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += NT) pre[i] = 0u;
    __syncthreads();
  }
}

// level 1: tile t of src into the bucket ranges of dst
template <int NT>
__global__ void __launch_bounds__(NT) k_jr_scatter(const unsigned long long* __restrict__ src,
                                                    const unsigned long long* hdr, uint64_t cap, uint32_t nb,
                                                    UDiv span, uint64_t nt, const uint64_t* __restrict__ offs,
                                                    unsigned long long* __restrict__ dst, uint32_t sub) {
  extern __shared__ unsigned long long smem64[];
  unsigned long long* srt = smem64;                                   // [sub] records by bucket
  uint64_t* run = reinterpret_cast<uint64_t*>(smem64 + sub);          // [nb] next position per bucket
  uint32_t* pre = reinterpret_cast<uint32_t*>(run + nb);              // [nb] counts, then prefix
  __shared__ uint32_t part[NT / 64];
  const uint64_t n = n_records(hdr, cap);
  uint64_t t;
  if (!xcd_tile(blockIdx.x, (n + kTile1 - 1) / kTile1, t)) return;
  const uint64_t a = t * kTile1;
  const uint64_t e = a + kTile1 < n ? a + kTile1 : n;
  for (uint32_t i = threadIdx.x; i < nb; i += NT) {
    run[i] = offs[(uint64_t)i * nt + t];
    pre[i] = 0u;
  }
  __syncthreads();
  scatter_range<NT>(src, a, e, 0, span, nb, run, pre, srt, part, dst, n, sub);
}

// level 2: tile k of coarse range c into its fpc buckets
template <int NT>
__global__ void __launch_bounds__(NT) k_jr_scatter2(const unsigned long long* __restrict__ src,
                                                     const unsigned long long* hdr, uint64_t cap, uint32_t fpc,
                                                     uint32_t nc, uint64_t nt, const uint64_t* __restrict__ offs1,
                                                     const uint32_t* __restrict__ tb,
                                                     const uint64_t* __restrict__ offs2, UDiv span,
                                                     unsigned long long* __restrict__ dst, uint32_t sub) {
  extern __shared__ unsigned long long smem64[];
  unsigned long long* srt = smem64;
  uint64_t* run = reinterpret_cast<uint64_t*>(smem64 + sub);
  uint32_t* pre = reinterpret_cast<uint32_t*>(run + fpc);
  __shared__ uint32_t part[NT / 64];
  uint64_t g;
  uint32_t c, k;
  if (!xcd_tile(blockIdx.x, tb[nc], g) || !tile2(tb, nc, (uint32_t)g, c, k)) return;
  const uint64_t n = n_records(hdr, cap);
  const uint64_t lo = offs1[(uint64_t)c * nt], hi = c + 1 < nc ? offs1[(uint64_t)(c + 1) * nt] : n;
  const uint64_t a = lo + (uint64_t)k * kTile1, e = a + kTile1 < hi ? a + kTile1 : hi;
  const uint32_t t0 = tb[c], ntc = tb[c + 1] - t0;
  for (uint32_t f = threadIdx.x; f < fpc; f += NT) {
    run[f] = offs2[(uint64_t)t0 * fpc + (uint64_t)f * ntc + k];
    pre[f] = 0u;
  }
  __syncthreads();
  scatter_range<NT>(src, a, e, (uint64_t)c * fpc * kBucketSlots, span, fpc, run, pre, srt, part, dst, n, sub);
}

// parts[b] = exclusive prefix of ceil(len_b / kPart) over buckets
__global__ void __launch_bounds__(1024) k_jr_items(const BucketMap M, unsigned long long* hdr, uint64_t cap,
                                                  uint32_t* __restrict__ parts) {
  __shared__ uint32_t s[1024];
  const uint64_t n = n_records(hdr, cap);
  const uint32_t nb = M.nb;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t b = b0; b < b0 + per && b < nb; ++b) {
    const uint64_t lo = bucket_start(M, b, n);
    const uint64_t hi = bucket_start(M, b + 1, n);
    loc += (uint32_t)((hi - lo + kPart - 1) / kPart);
  }
  s[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - loc;
  for (uint32_t b = b0; b < b0 + per && b < nb; ++b) {
    parts[b] = run;
    const uint64_t lo = bucket_start(M, b, n);
    const uint64_t hi = bucket_start(M, b + 1, n);
    run += (uint32_t)((hi - lo + kPart - 1) / kPart);
  }
  if (threadIdx.x == 1023) {
    parts[nb] = s[1023];
    hdr[1] = 0ull;
  }
}

__global__ void __launch_bounds__(1024) k_jr_sum(const unsigned long long* __restrict__ recB,
                                                unsigned long long* hdr, uint64_t cap, const BucketMap M,
                                                const uint32_t* __restrict__ parts, uint64_t n_slots,
                                                unsigned long long* __restrict__ jq) {
  extern __shared__ uint32_t acc[];
  __shared__ uint32_t s_item;
  const uint64_t n = n_records(hdr, cap);
  const uint32_t nb = M.nb;
  const uint32_t total = parts[nb];
  for (;;) {
    if (threadIdx.x == 0) s_item = (uint32_t)atomicAdd(&hdr[1], 1ull);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= total) break;
    uint32_t lo = 0, hi = nb;                       // bucket with parts[b] <= item < parts[b+1]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (parts[mid] <= item) lo = mid; else hi = mid;
    }
    const uint32_t b = lo;
    const uint64_t start = bucket_start(M, b, n);
    const uint64_t end = bucket_start(M, b + 1, n);
    const uint64_t r0 = start + (uint64_t)(item - parts[b]) * kPart;
    const uint64_t r1 = r0 + kPart < end ? r0 + kPart : end;
    const bool shared_bucket = parts[b + 1] - parts[b] > 1;
    const uint64_t base = (uint64_t)b * kBucketSlots;
    for (uint32_t i = threadIdx.x; i < kBucketSlots; i += 1024) acc[i] = 0u;
    __syncthreads();
    for (uint64_t k = r0 + threadIdx.x; k < r1; k += kLoads * 1024) {
      unsigned long long r[kLoads];
      // unconditional loads (past r1: record r0 again, dropped below): a
      // load under a branch makes the compiler wait for the earlier ones
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const uint64_t kk = k + (uint64_t)q * 1024;
        r[q] = recB[kk < r1 ? kk : r0];
      }
#pragma unroll
      for (int q = 0; q < kLoads; ++q) r[q] = k + (uint64_t)q * 1024 < r1 ? r[q] : 0ull;
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const uint64_t slot = r[q] >> kRecValBits;
        const uint32_t val = (uint32_t)(r[q] & kValMask);
        const uint64_t i = slot - base;
        if (val != 0u && i < kBucketSlots) {
          const uint32_t old = atomicAdd(&acc[i], val);
          if (old + val < old) atomicAdd(&jq[slot], 1ull << 32);
        }
      }
    }
    // this block's carry atomics complete before any of its threads reads the
    // words back below (no other block touches a single-item bucket, and a
    // shared bucket is written back by atomics only): a workgroup-scope fence
    // and the barrier, with each wave first waiting for its own memory
    // operations (vmcnt counts an atomic until the L2 acknowledges it).  An
    // agent-scope fence would also write back and invalidate the whole L2 of
    // the XCD, once per item.
    __threadfence_block();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const uint64_t ns = base >= n_slots ? 0 : (n_slots - base < kBucketSlots ? n_slots - base : kBucketSlots);
    for (uint32_t i0 = threadIdx.x; i0 < ns; i0 += 8 * 1024) {
      uint32_t v[8];
      unsigned long long old[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t i = i0 + q * 1024;
        v[q] = i < ns ? acc[i] : 0u;
      }
      if (shared_bucket) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (v[q]) atomicAdd(&jq[base + i0 + q * 1024], (unsigned long long)v[q]);
      } else {
        // the tally words' loads all in flight before the first store:
        // unconditional (past ns: word i0 again), since loads under a branch
        // make every store wait for all earlier memory operations
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t i = i0 + q * 1024;
          old[q] = jq[base + (i < ns ? i : i0)];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (v[q]) jq[base + i0 + q * 1024] = old[q] + v[q];
      }
    }
    __syncthreads();
  }
}

}  // namespace

JrecLayout jrec_layout(uint64_t n_slots, uint64_t capacity) {
  JrecLayout J{};
  J.capacity = capacity;
  J.n_buckets = (n_slots + kBucketSlots - 1) / kBucketSlots;
  J.n_tiles = (capacity + kTile1 - 1) / kTile1;
  J.two_level = J.n_buckets > kOneLevelMax;
  J.fpc = J.nc = 0;
  if (J.two_level) {
    uint64_t f = 1;
    while (f * f < J.n_buckets) ++f;
    J.fpc = f;
    J.nc = (J.n_buckets + f - 1) / f;
  }
  const uint64_t nb1 = J.two_level ? J.nc : J.n_buckets;
  const uint64_t nb_all = J.two_level ? J.nc * J.fpc : J.n_buckets;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += (bytes + 255) & ~255ull;
    return o;
  };
  J.hdr = take(64);
  J.counts = take(8 * nb1 * J.n_tiles);
  J.tb = take(4 * (J.nc + 1));
  J.counts2 = take(J.two_level ? 8 * (J.n_tiles + J.nc + 1) * J.fpc : 0);
  J.prefix = take(8 * (kScanBlocks + 1));
  J.parts = take(4 * (nb_all + 1));
  J.recA = take(8 * capacity);
  J.recB = take(8 * capacity);
  J.total = off;
  return J;
}

namespace {

__global__ void k_fill_u64(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

void scan_u64(uint64_t* v, uint64_t n, unsigned long long* bsum, hipStream_t s) {
  k_scan_sums<<<kScanBlocks, 256, 0, s>>>(v, n, bsum);
  k_scan_top<<<1, 64, 0, s>>>(bsum);
  k_scan_apply<<<kScanBlocks, 256, 0, s>>>(v, n, bsum);
}

// one scatter launch: one 1024-thread block per CU with the largest
// power-of-two sub-tile (<= 16384 records) whose sort buffer fits beside the
// two bucket arrays in 160 KB of LDS.  Longer sub-tiles mean longer runs of
// each bucket's stores, which pays more than two smaller blocks per CU
// overlapping their loads and sorts (7 % on the scatter of the flared disk).
template <typename L>
void scatter_launch(uint64_t nb, L launch) {
  uint32_t sub = 16384;
  while (sub > 1024 && (size_t)sub * 8 + 12 * nb + 256 > 160 * 1024) sub >>= 1;
  launch(sub, (size_t)sub * 8 + 12 * nb);
}

}  // namespace

hipError_t launch_jrec_accumulate(mcrt_ctx* c, const mcrt_run_opts& o, uint64_t* jq, hipStream_t s) {
  const uint64_t n_slots = (uint64_t)c->d.n_lambda * (uint64_t)c->d.n_cells;
  const JrecLayout J = jrec_layout(n_slots, o.jrec_capacity);
  unsigned char* ws = static_cast<unsigned char*>(o.jrec_ws);
  auto* hdr = reinterpret_cast<unsigned long long*>(ws + J.hdr);
  auto* counts = reinterpret_cast<uint64_t*>(ws + J.counts);
  auto* tb = reinterpret_cast<uint32_t*>(ws + J.tb);
  auto* counts2 = reinterpret_cast<uint64_t*>(ws + J.counts2);
  auto* bsum = reinterpret_cast<unsigned long long*>(ws + J.prefix);
  auto* parts = reinterpret_cast<uint32_t*>(ws + J.parts);
  auto* recA = reinterpret_cast<unsigned long long*>(ws + J.recA);
  auto* recB = reinterpret_cast<unsigned long long*>(ws + J.recB);
  auto* tally = reinterpret_cast<unsigned long long*>(jq);
  const uint64_t nt = J.n_tiles, cap = J.capacity;
  const uint32_t nb1 = (uint32_t)(J.two_level ? J.nc : J.n_buckets);
  const UDiv span1 = make_udiv((uint32_t)(J.two_level ? J.fpc * kBucketSlots : kBucketSlots));
  // level 1 (the whole partition for one level): recA -> recB
  const unsigned grid1 = (unsigned)((nt + kXcds - 1) / kXcds * kXcds);     // whole rounds over the XCDs
  k_jr_count<<<grid1, 256, 4 * (size_t)nb1, s>>>(recA, hdr, cap, nb1, span1, nt, counts);
  scan_u64(counts, (uint64_t)nb1 * nt, bsum, s);
  scatter_launch(nb1, [&](uint32_t sub, size_t lds) {
    k_jr_scatter<1024><<<grid1, 1024, lds, s>>>(recA, hdr, cap, nb1, span1, nt, counts, recB, sub);
  });
  BucketMap M{};
  const unsigned long long* sorted = recB;
  if (!J.two_level) {
    M.offs = counts; M.tb = nullptr; M.nt = nt; M.nb = nb1;
  } else {
    // level 2: each coarse range of recB, tile by tile, into its buckets -> recA
    const uint32_t fpc = (uint32_t)J.fpc, nc = (uint32_t)J.nc;
    const uint64_t n2 = (nt + nc + 1) * fpc;
    const unsigned grid2 = (unsigned)((nt + nc + kXcds - 1) / kXcds * kXcds);  // >= level-2 tiles
    k_jr_dir<<<1, 1024, 0, s>>>(counts, hdr, cap, nc, nt, tb);
    k_fill_u64<<<256, 256, 0, s>>>(counts2, n2);
    const UDiv span2 = make_udiv((uint32_t)kBucketSlots);
    k_jr_count2<<<grid2, 256, 4 * (size_t)fpc, s>>>(recB, hdr, cap, fpc, nc, nt, counts, tb, span2, counts2);
    scan_u64(counts2, n2, bsum, s);
    scatter_launch(fpc, [&](uint32_t sub, size_t lds) {
      k_jr_scatter2<1024><<<grid2, 1024, lds, s>>>(recB, hdr, cap, fpc, nc, nt, counts, tb, counts2, span2, recA, sub);
    });
    M.offs = counts2; M.tb = tb; M.nt = nt; M.fpc = fpc; M.nc = nc; M.nb = nc * fpc;
    sorted = recA;
  }
  k_jr_items<<<1, 1024, 0, s>>>(M, hdr, cap, parts);
  k_jr_sum<<<(unsigned)c->n_cu, 1024, 4 * kBucketSlots, s>>>(sorted, hdr, cap, M, parts, n_slots, tally);
  return hipGetLastError();
}

}  // namespace mcrt

extern "C" int32_t mcrt_jrec_ws_bytes(const mcrt_ctx* ctx, uint64_t capacity, uint64_t* bytes) {
  if (!ctx || !bytes) return MCRT_E_INVALID;
  const uint64_t n_slots = (uint64_t)ctx->d.n_lambda * (uint64_t)ctx->d.n_cells;
  if (capacity < mcrt::kRecChunk || capacity > mcrt::kMaxRecords) return MCRT_E_INVALID;
  if (ctx->d.max_level > 7 || n_slots >= (1ull << 40)) return MCRT_E_UNSUPPORTED;
  const mcrt::JrecLayout J = mcrt::jrec_layout(n_slots, capacity);
  const uint64_t nb1 = J.two_level ? J.nc : J.n_buckets;
  if (J.n_buckets > mcrt::kMaxBuckets || nb1 * J.n_tiles > (1ull << 26) ||
      (J.two_level && (J.n_tiles + J.nc + 1) * J.fpc > (1ull << 26)))
    return MCRT_E_UNSUPPORTED;
  *bytes = J.total;
  return MCRT_OK;
}
