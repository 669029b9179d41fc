// Deferred path-length tally (the mean-intensity estimator of Lucy 1999 that
// the paper's method accumulates per cell and wavelength).  Random 64-bit
// atomics into the tally are limited by the L2 atomic units whatever the
// table size, so the transport instead appends one record per path segment,
// (tally index << 24) | fixed-point length, contiguously per wave.  Here the
// records are added to the tally with streaming passes and LDS sums:
//   plan     every bucket (kBucketSlots tally words) gets a region of the
//            destination array: its exact record count for the first id
//            range of a chain of consecutive ranges (a counting pass), else
//            the previous range's total (plus its growth over the range
//            before that, if it grew) scaled to this range's records, plus
//            kPad records and a share of the array's room left in proportion
//            to it; regions that would not fit the array are shrunk in
//            proportion
//   scatter  records to their bucket regions (sub-tiles sorted in LDS first);
//            each sub-tile claims its run of every bucket with one atomic add
//            on that bucket's fill counter, and the records past the end of a
//            region are added to the tally directly (atomic adds)
//   items    work items of at most kPart records per bucket
//   sum      per item, u32 partial sums of its bucket (kBucketSlots tally
//            words) in LDS (a carry past 2^32 goes straight to the tally),
//            then one add per tally word: plain for a bucket of one item,
//            atomic for a bucket shared by several items.
// A tally of many buckets is partitioned in two levels, so that every
// scatter writes long runs: first into coarse ranges of fpc buckets, then
// each coarse range, tile by tile, into its buckets.
// Integer sums do not depend on order, so the tally equals the one the
// atomic path gives, bit for bit, whichever records overflow their regions.
#include "mcrt_internal.h"

namespace mcrt {

namespace {

constexpr uint64_t kPart = 1ull << 20;      // records per summing work item
constexpr int kLoads = 16;                  // record loads per thread in flight (counting passes, sum)
constexpr unsigned long long kValMask = (1ull << kRecValBits) - 1ull;
constexpr uint64_t kPad = 1024;
// records per level-2 tile: the blocks resident at once then span fewer
// coarse ranges, and so fewer bucket regions take writes at a time (2^16
// against 2^18: the level-2 scatter 1.6 % faster on the 256^3 disk)
constexpr uint64_t kTile2 = 1ull << 16;             // records added to every estimated region
// A scatter block has 512 threads (two blocks per CU, up to 806 buckets) or
// 1024 (one per CU); each thread claims for at most two buckets: one level
// has at most kOneLevelMax buckets, two levels at most 1024 per range
static_assert(kOneLevelMax <= 2 * 1024 && kMaxBuckets <= 1024 * 1024, "bucket counts per scatter block");

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

// bucket of a record among nb buckets of D.d tally words from slot0; WIDE
// for a tally of 2^32 words or more (else the offset always fits 32 bits,
// and the kernel has no 64-bit division to hold registers for)
template <bool WIDE = true>
__device__ __forceinline__ uint32_t bucket_of(unsigned long long r, uint64_t slot0, const UDiv& D, uint32_t nb) {
  const uint64_t slot = r >> kRecValBits;
  const uint64_t d = slot >= slot0 ? slot - slot0 : 0;
  const uint64_t b = !WIDE || d < (1ull << 32) ? (uint64_t)udiv((uint32_t)d, D) : d / D.d;
  return b < nb ? (uint32_t)b : nb - 1;
}

// The regions of one partition level's nb buckets in its destination array:
// est[b] the record total a region is sized from (one more word after the
// level-1 totals: the records they stand for), start[b] and size[b] the
// region, fill[b] its next free place (start[b] plus the records claimed so
// far: the exact total once the scatter is done, overflow included), prev[b]
// the total of the range before.
struct Level {
  unsigned long long* est;
  unsigned long long* fill;
  uint64_t* start;
  uint64_t* size;
  unsigned long long* prev;
  uint32_t nb;
};

// records a bucket's region holds after the scatter
__device__ __forceinline__ uint64_t filled(const Level& L, uint32_t b) {
  const uint64_t f = L.fill[b] - L.start[b], z = L.size[b];
  return f < z ? f : z;
}

// Barrier for LDS hazards only: fences limited to the local address space,
// so a wave does not first wait for its global loads and stores in flight
// (__syncthreads does).  The scatter's threads share nothing but LDS, and its
// next sub-tile's loads then overlap the stores of the previous one.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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
// contiguous range of tiles: the level-2 tiles of one coarse range then run
// on one XCD, whose L2 completes the cache lines where their runs of a bucket
// meet and takes the atomics on that range's fill counters.  The grid needs
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

// Exact record totals of the first range of a chain, level 1: tile t of the
// record array counted in LDS, then one atomic add per bucket into est.
__global__ void __launch_bounds__(256) k_jr_total(const unsigned long long* __restrict__ rec,
                                                 const unsigned long long* hdr, uint64_t cap, uint32_t nb,
                                                 UDiv span, unsigned long long* __restrict__ est) {
  extern __shared__ uint32_t h[];
  const uint64_t n = n_records(hdr, cap);
  uint64_t t;
  if (!xcd_tile(blockIdx.x, (n + kTile1 - 1) / kTile1, t)) return;
  for (uint32_t i = threadIdx.x; i < nb; i += 256) h[i] = 0u;
  __syncthreads();
  const uint64_t a = t * kTile1, e = a + kTile1 < n ? a + kTile1 : n;
  count_range(rec, a, e, 0, span, nb, h);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nb; i += 256)
    if (h[i]) atomicAdd(&est[i], (unsigned long long)h[i]);
}

// Block-wide exclusive scan of one u64 per thread (1024 threads): shuffles
// within each wave, the 16 wave totals through part (LDS).  Returns the
// thread's exclusive prefix; *total gets the block's sum.  Two barriers.
__device__ __forceinline__ uint64_t scan1024(uint64_t x, uint64_t* part, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t inc = x;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63u) part[wave] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (uint32_t w = 0; w < 16; ++w) {
    const uint64_t t = part[w];
    before += w < wave ? t : 0ull;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// Regions of one level (one block).  Exact totals are the sizes as they
// are.  Estimates are scaled by n / est_n (this range's records over those
// they were taken from) and given kPad records each, and the space left in
// the destination (`space` records) is dealt out in proportion to them: the
// totals of one bucket vary by tens of percent from range to range (a few
// packets that scatter many times in thick cells leave most of some cells'
// records).  Regions that would not fit are shrunk in proportion (and by one
// record against rounding).  Records past a region's end are still added
// exactly.  Sets the fill counters to the region starts.
__global__ void __launch_bounds__(1024) k_jr_plan(const unsigned long long* hdr, uint64_t cap, Level L,
                                                 const unsigned long long* est_n, int exact, uint64_t space) {
  __shared__ uint64_t part[16];
  const uint64_t n = n_records(hdr, cap);
  const uint32_t nb = L.nb;
  const uint64_t en = exact ? 0 : *est_n;
  const double f = en ? (double)n / (double)en : 0.0;
  // each base at most `space`, so that no sum below can wrap whatever the
  // workspace holds (a workspace reallocated at the same address leaves
  // arbitrary estimates: they cost speed, never bounds)
  auto base = [&](uint32_t b) -> uint64_t {
    if (b >= nb) return 0;
    const uint64_t x = L.est[b];
    return exact ? (x < space ? x : space) : (uint64_t)fmin((double)x * f, (double)space) + 1;
  };
  // chunks of 1024 consecutive buckets, one per thread
  uint64_t W = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += 1024) {
    uint64_t t;
    scan1024(base(c0 + threadIdx.x), part, &t);
    W += t;
  }
  const uint64_t pad = exact ? 0 : kPad, pads = (uint64_t)nb * pad;
  // sizes: exact; base + kPad + a share of the room left; or, when they would
  // not fit, shrunk in proportion (W + pads <= 2^56: no wrap)
  const int mode = W + pads <= space ? (exact ? 0 : 1) : 2;
  const double g = mode == 1 ? (double)(space - W - pads) / (double)W : (double)space / (double)(W + pads);
  auto size = [&](uint32_t b) -> uint64_t {
    if (b >= nb) return 0;
    const uint64_t w = base(b);
    if (mode == 0) return w;
    if (mode == 1) {
      const uint64_t x = (uint64_t)((double)w * g);
      return w + pad + (x ? x - 1 : 0);
    }
    const uint64_t x = (uint64_t)((double)(w + pad) * g);
    return x ? x - 1 : 0;
  };
  uint64_t carry = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += 1024) {
    const uint32_t b = c0 + threadIdx.x;
    const uint64_t z = size(b);
    uint64_t t;
    const uint64_t at = carry + scan1024(z, part, &t);
    if (b < nb) {
      L.start[b] = at;
      L.size[b] = z;
      L.fill[b] = at;
    }
    carry += t;
  }
}

// level-2 tiles of each coarse range: tb[c] = tiles before range c (the
// records its level-1 region holds), tb[nc] = all tiles
__global__ void __launch_bounds__(1024) k_jr_dir(const Level L1, uint32_t nc, uint32_t* __restrict__ tb) {
  __shared__ uint32_t s[1024];
  const uint32_t per = (nc + 1023) / 1024, c0 = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t c = c0; c < c0 + per && c < nc; ++c) loc += (uint32_t)((filled(L1, c) + kTile2 - 1) / kTile2);
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
    run += (uint32_t)((filled(L1, c) + kTile2 - 1) / kTile2);
  }
  if (threadIdx.x == 1023) tb[nc] = s[1023];
}

// records [a, e) of level-2 tile g (tile k of coarse range c's region)
__device__ __forceinline__ bool tile2_range(const uint32_t* tb, uint32_t nc, uint64_t g, const Level& L1,
                                            uint32_t& c, uint64_t& a, uint64_t& e) {
  uint32_t k;
  if (!tile2(tb, nc, (uint32_t)g, c, k)) return false;
  const uint64_t lo = L1.start[c], hi = lo + filled(L1, c);
  a = lo + (uint64_t)k * kTile2;
  e = a + kTile2 < hi ? a + kTile2 : hi;
  return true;
}

// Exact record totals, level 2: level-2 tile g counted over the fpc buckets
// of its coarse range c, one atomic add per bucket into est.
__global__ void __launch_bounds__(256) k_jr_total2(const unsigned long long* __restrict__ rec, uint32_t fpc,
                                                  uint32_t nc, const Level L1, const uint32_t* __restrict__ tb,
                                                  UDiv span, unsigned long long* __restrict__ est) {
  extern __shared__ uint32_t h[];
  uint64_t g, a, e;
  uint32_t c;
  if (!xcd_tile(blockIdx.x, tb[nc], g) || !tile2_range(tb, nc, g, L1, c, a, e)) return;
  for (uint32_t i = threadIdx.x; i < fpc; i += 256) h[i] = 0u;
  __syncthreads();
  count_range(rec, a, e, (uint64_t)c * fpc * kBucketSlots, span, fpc, h);
  __syncthreads();
  for (uint32_t f = threadIdx.x; f < fpc; f += 256)
    if (h[f]) atomicAdd(&est[(uint64_t)c * fpc + f], (unsigned long long)h[f]);
}

// Block-wide exclusive scan of v[0, n) in LDS with NT threads; returns the
// total.  Each thread sums its run of entries, the runs are scanned within
// each wave by shuffles and across the NT / 64 waves through part (LDS
// scratch of NT / 64 words): two barriers in all (LDS only).
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
  lds_barrier();
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
  lds_barrier();
  return total;
}

// The records [a, e) of src, sub-tile by sub-tile sorted by bucket in LDS
// and written as contiguous runs (consecutive threads, consecutive
// addresses) into the buckets' regions of dst.  Each sub-tile claims the run
// of each of its buckets with one atomic add on the bucket's fill counter
// (fill[b], the next free place); a record whose place falls past its
// region's end (lim[b]) is added to the tally jq directly, and counted in
// ovf.  Thread i claims for buckets i, i + NT, ... (OWN of them, nb <= OWN NT).
// LDS: srt [sub] records, run [nb] place of the sub-tile's run per bucket,
// lim [nb], pre [nb] counts, then their prefix.
template <int NT, int OWN, bool WIDE>
__device__ void scatter_range(const unsigned long long* __restrict__ src, uint64_t a, uint64_t e, uint64_t slot0,
                              const UDiv& span, uint32_t nb, unsigned long long* fill, uint64_t* run,
                              const uint64_t* lim, uint32_t* pre, unsigned long long* srt, uint32_t* part,
                              unsigned long long* __restrict__ dst, unsigned long long* __restrict__ jq,
                              uint64_t n_slots, uint32_t sub, uint32_t& ovf) {
  constexpr int kMaxPer = 16;                                         // sub <= 16 NT
  for (uint64_t s0 = a; s0 < e; s0 += sub) {
    const uint32_t m = (uint32_t)(e - s0 < sub ? e - s0 : sub);
    unsigned long long r[kMaxPer];
    uint32_t br[kMaxPer];                     // bucket << 16 | rank in the bucket (nb <= 2048, sub <= 16384)
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
      const uint32_t b = bucket_of<WIDE>(r[q], slot0, span, nb);
      br[q] = b << 16 | (k < m ? atomicAdd(&pre[b], 1u) : 0u);
    }
    lds_barrier();
    // claim the runs; their places are first needed after the LDS sort
    unsigned long long got[OWN];
#pragma unroll
    for (int j = 0; j < OWN; ++j) {
      const uint32_t i = threadIdx.x + (uint32_t)j * NT;
      const uint32_t cnt = i < nb ? pre[i] : 0u;
      got[j] = cnt ? atomicAdd(&fill[i], (unsigned long long)cnt) : ~0ull;
    }
    block_exclusive_scan<NT>(pre, nb, part);
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      if (k < m) srt[pre[br[q] >> 16] + (br[q] & 0xffffu)] = r[q];
    }
#pragma unroll
    for (int j = 0; j < OWN; ++j)
      if (got[j] != ~0ull) run[threadIdx.x + (uint32_t)j * NT] = got[j];
    lds_barrier();
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      // in two halves: the LDS reads of all sixteen at once would not fit
      // the registers of four waves per SIMD
      if (q == kMaxPer / 2) __builtin_amdgcn_sched_barrier(0);
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      const uint32_t kk = k < m ? k : 0u;
      const unsigned long long x = srt[kk];
      const uint32_t b = bucket_of<WIDE>(x, slot0, span, nb);
      const uint64_t d = run[b] + (kk - pre[b]);
      // plain store: a bucket's runs are completed across sub-tiles in the L2
      // (non-temporal stores made this pass 23 % slower)
      if (k < m) {
        if (d < lim[b]) {
          dst[d] = x;
        } else {
          const uint64_t slot = x >> kRecValBits;
          const unsigned long long val = x & kValMask;
          if (val && slot < n_slots) atomicAdd(&jq[slot], val);
          ++ovf;
        }
      }
    }
    lds_barrier();
    for (uint32_t i = threadIdx.x; i < nb; i += NT) pre[i] = 0u;
    lds_barrier();
  }
}

// LDS of a scatter block: the sort buffer and the three bucket arrays
constexpr size_t scatter_lds(uint32_t sub, uint64_t nb) { return (size_t)sub * 8 + 20 * nb; }

// region ends of buckets [b0, b0 + nb) of L into LDS
template <int NT>
__device__ __forceinline__ void scatter_setup(const Level& L, uint32_t b0, uint32_t nb, uint64_t* lim, uint32_t* pre) {
  for (uint32_t i = threadIdx.x; i < nb; i += NT) {
    lim[i] = L.start[b0 + i] + L.size[b0 + i];
    pre[i] = 0u;
  }
  __syncthreads();
}

// level 1: tile t of src into the regions of L's buckets in dst
template <int NT, int OWN, bool WIDE>
__global__ void __launch_bounds__(NT, 4) k_jr_scatter(const unsigned long long* __restrict__ src,
                                                       unsigned long long* hdr, uint64_t cap, UDiv span, const Level L,
                                                    unsigned long long* __restrict__ dst,
                                                    unsigned long long* __restrict__ jq, uint64_t n_slots,
                                                    uint32_t sub) {
  extern __shared__ unsigned long long smem64[];
  const uint32_t nb = L.nb;
  unsigned long long* srt = smem64;
  uint64_t* run = reinterpret_cast<uint64_t*>(smem64 + sub);
  uint64_t* lim = run + nb;
  uint32_t* pre = reinterpret_cast<uint32_t*>(lim + nb);
  __shared__ uint32_t part[NT / 64];
  const uint64_t n = n_records(hdr, cap);
  uint64_t t;
  if (!xcd_tile(blockIdx.x, (n + kTile1 - 1) / kTile1, t)) return;
  const uint64_t a = t * kTile1;
  const uint64_t e = a + kTile1 < n ? a + kTile1 : n;
  scatter_setup<NT>(L, 0, nb, lim, pre);
  uint32_t ovf = 0;
  scatter_range<NT, OWN, WIDE>(src, a, e, 0, span, nb, L.fill, run, lim, pre, srt, part, dst, jq, n_slots, sub, ovf);
  if (ovf) atomicAdd(&hdr[2], (unsigned long long)ovf);
}

// level 2: level-2 tile g (tile k of coarse range c's region in src) into the
// regions of c's fpc buckets of L2 in dst
template <int NT, int OWN, bool WIDE>
__global__ void __launch_bounds__(NT, 4) k_jr_scatter2(const unsigned long long* __restrict__ src,
                                                        unsigned long long* hdr, uint32_t fpc, uint32_t nc,
                                                        const Level L1,
                                                     const uint32_t* __restrict__ tb, const Level L2, UDiv span,
                                                     unsigned long long* __restrict__ dst,
                                                     unsigned long long* __restrict__ jq, uint64_t n_slots,
                                                     uint32_t sub) {
  extern __shared__ unsigned long long smem64[];
  unsigned long long* srt = smem64;
  uint64_t* run = reinterpret_cast<uint64_t*>(smem64 + sub);
  uint64_t* lim = run + fpc;
  uint32_t* pre = reinterpret_cast<uint32_t*>(lim + fpc);
  __shared__ uint32_t part[NT / 64];
  uint64_t g, a, e;
  uint32_t c;
  if (!xcd_tile(blockIdx.x, tb[nc], g) || !tile2_range(tb, nc, g, L1, c, a, e)) return;
  const uint32_t b0 = c * fpc;
  scatter_setup<NT>(L2, b0, fpc, lim, pre);
  uint32_t ovf = 0;
  scatter_range<NT, OWN, WIDE>(src, a, e, (uint64_t)b0 * kBucketSlots, span, fpc, L2.fill + b0, run, lim, pre, srt,
                               part, dst, jq, n_slots, sub, ovf);
  if (ovf) atomicAdd(&hdr[2], (unsigned long long)ovf);
}

// The estimate of a bucket for the next range from its total t of this one
// and p of the one before (counted over n and n_prev records): t plus the
// growth since, if it grew.  Over a pass the totals drift (re-emission
// follows the dust temperatures, which rise as absorptions are counted), by
// tens of percent between the first ranges.
__device__ __forceinline__ uint64_t next_estimate(uint64_t t, uint64_t p, uint64_t n, uint64_t n_prev, bool first) {
  if (first || !n_prev) return t;
  const double grow = (double)t - (double)p * ((double)n / (double)n_prev);
  return grow > 0.0 ? t + (uint64_t)grow : t;
}

// parts[b] = exclusive prefix of ceil(len_b / kPart) over the buckets of M
// (the last level); then the next range's estimates of both levels (L1 and M,
// the same level for one level), with est_n = n; `first`: the first range of
// a chain (no totals before).  With two levels (fpc > 0), a coarse range's
// records that did not fit its level-1 region never reached level 2: its
// buckets' totals are scaled up by the coarse range's total over the records
// its region held.
__global__ void __launch_bounds__(1024) k_jr_items(const Level M, const Level L1, uint32_t fpc, int first,
                                                  unsigned long long* hdr, uint64_t cap,
                                                  uint32_t* __restrict__ parts) {
  __shared__ uint64_t part[16];
  const uint64_t n = n_records(hdr, cap);
  const uint64_t n_prev = first ? 0 : L1.est[L1.nb];     // read by all before the barriers below
  const uint32_t nb = M.nb;
  uint64_t carry = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += 1024) {           // chunks of consecutive buckets
    const uint32_t b = c0 + threadIdx.x;
    uint64_t x = 0;
    if (b < nb) {
      x = (filled(M, b) + kPart - 1) / kPart;
      uint64_t t = M.fill[b] - M.start[b];
      if (fpc) {
        const uint32_t c = b / fpc;
        const uint64_t t1 = L1.fill[c] - L1.start[c], h1 = filled(L1, c);
        if (t1 > h1 && h1) t = (uint64_t)((double)t * (double)t1 / (double)h1);
      }
      M.est[b] = next_estimate(t, M.prev[b], n, n_prev, first);
      M.prev[b] = t;
    }
    uint64_t tot;
    const uint64_t ex = scan1024(x, part, &tot);
    if (b < nb) parts[b] = (uint32_t)(carry + ex);
    carry += tot;
  }
  if (fpc) {
    for (uint32_t c = threadIdx.x; c < L1.nb; c += 1024) {
      const uint64_t t = L1.fill[c] - L1.start[c];
      L1.est[c] = next_estimate(t, L1.prev[c], n, n_prev, first);
      L1.prev[c] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    parts[nb] = (uint32_t)carry;
    L1.est[L1.nb] = n;
    hdr[1] = 0ull;
  }
}

__global__ void __launch_bounds__(1024) k_jr_sum(const unsigned long long* __restrict__ recB,
                                                unsigned long long* hdr, const Level M,
                                                const uint32_t* __restrict__ parts, uint64_t n_slots,
                                                unsigned long long* __restrict__ jq) {
  extern __shared__ uint32_t acc[];
  __shared__ uint32_t s_item;
  const uint32_t nb = M.nb;
  const uint32_t total = parts[nb];
  for (;;) {
    if (threadIdx.x == 0) s_item = (uint32_t)atomicAdd(&hdr[1], 1ull);
    lds_barrier();
    const uint32_t item = s_item;
    lds_barrier();
    if (item >= total) break;
    uint32_t lo = 0, hi = nb;                       // bucket with parts[b] <= item < parts[b+1]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (parts[mid] <= item) lo = mid; else hi = mid;
    }
    const uint32_t b = lo;
    const uint64_t start = M.start[b];
    const uint64_t end = start + filled(M, b);
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
    const __amdgpu_buffer_rsrc_t words =
        __builtin_amdgcn_make_buffer_rsrc(jq + base, (short)0, (int)(8 * ns), 0x00020000);
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
        // the tally words' loads all in flight before the first store, with
        // no branch (a load under a branch makes every store wait for all
        // earlier memory operations): buffer loads over the bucket's words,
        // whose offset is out of range for a word this item adds nothing to
        // (such a load reads no memory and returns 0; a range adds to about
        // a third of the words)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t i = i0 + q * 1024;
          old[q] = __builtin_bit_cast(unsigned long long,
                                      __builtin_amdgcn_raw_buffer_load_b64(words, v[q] ? 8u * i : 0xffffffffu, 0, 0));
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (v[q]) jq[base + i0 + q * 1024] = old[q] + v[q];
      }
    }
    // LDS only: the next item's loads overlap this item's write-back (no
    // other item writes these tally words but by atomics)
    lds_barrier();
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
  J.tb = take(4 * (J.nc + 1));
  J.parts = take(4 * (nb_all + 1));
  J.lvl1 = take(8 * (5 * nb1 + 1));                     // est [nb1 + 1], fill, start, size, prev
  J.lvl2 = take(J.two_level ? 8 * 5 * nb_all : 0);     // est, fill, start, size, prev
  J.recA = take(8 * capacity);
  J.recB = take(8 * capacity);
  J.total = off;
  return J;
}

namespace {

__global__ void k_fill_u64(unsigned long long* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

Level level_at(unsigned char* base, uint64_t nb, uint64_t est_words) {
  Level L{};
  auto* w = reinterpret_cast<unsigned long long*>(base);
  L.est = w;
  L.fill = w + est_words;
  L.start = reinterpret_cast<uint64_t*>(L.fill + nb);
  L.size = L.start + nb;
  L.prev = reinterpret_cast<unsigned long long*>(L.size + nb);
  L.nb = (uint32_t)nb;
  return L;
}

// One scatter launch (each thread at most 128 registers, 16 records per
// sub-tile).  Where sub-tiles of 8192 records fit two blocks' LDS (160 KB per
// CU; up to 806 buckets), two 512-thread blocks per CU: one block's LDS sort
// then overlaps the other's loads and stores.  On the 256^3 disk the level-1
// scatter takes 21 % less time than one 1024-thread block per CU on
// sub-tiles of 16384 records; four 256-thread blocks on 4096 take 30 % more
// (a bucket's runs get too short).  More buckets: one 1024-thread block per
// CU with the largest power-of-two sub-tile (<= 16384) that fits.
template <typename F>
void scatter_launch(uint64_t nb, F launch) {
  if (2 * (scatter_lds(8192, nb) + 256) <= 160 * 1024) {
    launch(512, 8192u, scatter_lds(8192, nb));
    return;
  }
  uint32_t sub = 16384;
  while (sub > 1024 && scatter_lds(sub, nb) + 256 > 160 * 1024) sub >>= 1;
  launch(1024, sub, scatter_lds(sub, nb));
}

template <int NT, int OWN>
auto scatter1_kernel(bool wide) { return wide ? k_jr_scatter<NT, OWN, true> : k_jr_scatter<NT, OWN, false>; }
template <int NT, int OWN>
auto scatter2_kernel(bool wide) { return wide ? k_jr_scatter2<NT, OWN, true> : k_jr_scatter2<NT, OWN, false>; }

}  // namespace

hipError_t launch_jrec_accumulate(mcrt_ctx* c, const mcrt_run_opts& o, uint64_t first_id, uint64_t n_packets,
                                  uint64_t* jq, hipStream_t s) {
  const uint64_t n_slots = (uint64_t)c->d.n_lambda * (uint64_t)c->d.n_cells;
  const JrecLayout J = jrec_layout(n_slots, o.jrec_capacity);
  unsigned char* ws = static_cast<unsigned char*>(o.jrec_ws);
  auto* hdr = reinterpret_cast<unsigned long long*>(ws + J.hdr);
  auto* tb = reinterpret_cast<uint32_t*>(ws + J.tb);
  auto* parts = reinterpret_cast<uint32_t*>(ws + J.parts);
  auto* recA = reinterpret_cast<unsigned long long*>(ws + J.recA);
  auto* recB = reinterpret_cast<unsigned long long*>(ws + J.recB);
  auto* tally = reinterpret_cast<unsigned long long*>(jq);
  const uint64_t nt = J.n_tiles, cap = J.capacity;
  const uint32_t nb1 = (uint32_t)(J.two_level ? J.nc : J.n_buckets);
  const Level L1 = level_at(ws + J.lvl1, nb1, nb1 + 1);
  // a range that continues the last one of this context on the same
  // workspace (same capacity, seed and pass size, the next packet ids) is the
  // next of a chain; the first of a chain counts its records, the others size
  // their regions from the totals of the ranges before.  The second range,
  // with no growth to go by, leaves a few percent of its records past their
  // regions where the totals drift; those direct adds cost far less than a
  // counting pass per level (on the 128^3 disk's two ranges: 263 against
  // 277 ms per pass).
  JrecChain& ch = c->jchain;
  const bool chained = ch.ws == o.jrec_ws && ch.capacity == cap && ch.seed == o.seed && ch.n_total == o.n_total &&
                       ch.next_id == first_id;
  const uint64_t ch_len = chained ? ch.length : 0;
  const bool exact = ch_len < 1;
  ch = JrecChain{};
  const UDiv span1 = make_udiv((uint32_t)(J.two_level ? J.fpc * kBucketSlots : kBucketSlots));
  // level 1 (the whole partition for one level): recA -> recB
  const unsigned grid1 = (unsigned)((nt + kXcds - 1) / kXcds * kXcds);     // whole rounds over the XCDs
  if (exact) {
    k_fill_u64<<<64, 256, 0, s>>>(L1.est, nb1);
    k_jr_total<<<grid1, 256, 4 * (size_t)nb1, s>>>(recA, hdr, cap, nb1, span1, L1.est);
  }
  k_jr_plan<<<1, 1024, 0, s>>>(hdr, cap, L1, L1.est + nb1, exact ? 1 : 0, cap);
  const bool wide = n_slots > (1ull << 32);
  scatter_launch(nb1, [&](int nt, uint32_t sub, size_t lds) {
    const bool two = nb1 > (uint32_t)nt;                       // buckets per thread
    auto k = nt == 512 ? (two ? scatter1_kernel<512, 2>(wide) : scatter1_kernel<512, 1>(wide))
                       : (two ? scatter1_kernel<1024, 2>(wide) : scatter1_kernel<1024, 1>(wide));
    k<<<grid1, nt, lds, s>>>(recA, hdr, cap, span1, L1, recB, tally, n_slots, sub);
  });
  Level M = L1;
  const unsigned long long* sorted = recB;
  if (J.two_level) {
    // level 2: each coarse range of recB, tile by tile, into its buckets -> recA
    const uint32_t fpc = (uint32_t)J.fpc, nc = (uint32_t)J.nc;
    const uint64_t nb2 = (uint64_t)nc * fpc;
    const Level L2 = level_at(ws + J.lvl2, nb2, nb2);
    const uint64_t nt2 = (cap + kTile2 - 1) / kTile2;
    const unsigned grid2 = (unsigned)((nt2 + nc + kXcds - 1) / kXcds * kXcds);  // >= level-2 tiles
    const UDiv span2 = make_udiv((uint32_t)kBucketSlots);
    k_jr_dir<<<1, 1024, 0, s>>>(L1, nc, tb);
    if (exact) {
      k_fill_u64<<<256, 256, 0, s>>>(L2.est, nb2);
      k_jr_total2<<<grid2, 256, 4 * (size_t)fpc, s>>>(recB, fpc, nc, L1, tb, span2, L2.est);
    }
    k_jr_plan<<<1, 1024, 0, s>>>(hdr, cap, L2, L1.est + nb1, exact ? 1 : 0, cap);
    scatter_launch(fpc, [&](int nt, uint32_t sub, size_t lds) {
      const bool two = fpc > (uint32_t)nt;
      auto k = nt == 512 ? (two ? scatter2_kernel<512, 2>(wide) : scatter2_kernel<512, 1>(wide))
                         : (two ? scatter2_kernel<1024, 2>(wide) : scatter2_kernel<1024, 1>(wide));
      k<<<grid2, nt, lds, s>>>(recB, hdr, fpc, nc, L1, tb, L2, span2, recA, tally, n_slots, sub);
    });
    M = L2;
    sorted = recA;
  }
  k_jr_items<<<1, 1024, 0, s>>>(M, L1, J.two_level ? (uint32_t)J.fpc : 0u, ch_len == 0 ? 1 : 0, hdr, cap, parts);
  k_jr_sum<<<(unsigned)c->n_cu, 1024, 4 * kBucketSlots, s>>>(sorted, hdr, M, parts, n_slots, tally);
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) ch = JrecChain{o.jrec_ws, cap, o.seed, o.n_total, first_id + n_packets, ch_len + 1};
  return e;
}

}  // namespace mcrt

extern "C" int32_t mcrt_jrec_ws_bytes(const mcrt_ctx* ctx, uint64_t capacity, uint64_t* bytes) {
  if (!ctx || !bytes) return MCRT_E_INVALID;
  const uint64_t n_slots = (uint64_t)ctx->d.n_lambda * (uint64_t)ctx->d.n_cells;
  if (capacity < mcrt::kRecChunk || capacity > mcrt::kMaxRecords) return MCRT_E_INVALID;
  if (ctx->d.max_level > 7 || n_slots >= (1ull << 40)) return MCRT_E_UNSUPPORTED;
  const mcrt::JrecLayout J = mcrt::jrec_layout(n_slots, capacity);
  if (J.n_buckets > mcrt::kMaxBuckets) return MCRT_E_UNSUPPORTED;
  *bytes = J.total;
  return MCRT_OK;
}
