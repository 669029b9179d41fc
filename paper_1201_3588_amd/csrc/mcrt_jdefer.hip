// Deferred path-length tally (the mean-intensity estimator of Lucy 1999 that
// the paper's method accumulates per cell and wavelength).  Random 64-bit
// atomics into the tally are limited by the L2 atomic units whatever the
// table size, so the transport instead appends one record per path segment,
// (tally index << 24) | fixed-point length, contiguously per wave.  Here the
// records are added to the tally with streaming passes and LDS sums:
//   count    histogram of records per (bucket of kBucketSlots tally words, tile)
//   scan     exclusive scan of the counts, bucket-major: each bucket's records
//            become one contiguous range, ordered by tile
//   scatter  records to their bucket ranges
//   items    work items of at most kPart records per bucket
//   sum      per item, u32 partial sums of its bucket in LDS (a carry past
//            2^32 goes straight to the tally), then one add per tally word:
//            plain for a bucket of one item, atomic for a bucket shared by
//            several items.
// Integer sums do not depend on order, so the tally equals the one the
// atomic path gives, bit for bit.
#include "mcrt_internal.h"

namespace mcrt {

namespace {

constexpr int kScanBlocks = 256;
constexpr uint64_t kPart = 1ull << 20;      // records per summing work item
constexpr unsigned long long kValMask = (1ull << kRecValBits) - 1ull;

__device__ __forceinline__ uint32_t bucket_of(unsigned long long r, uint32_t nb) {
  const uint64_t b = (r >> kRecValBits) / kBucketSlots;
  return b < nb ? (uint32_t)b : nb - 1;
}

__device__ __forceinline__ uint64_t n_records(const unsigned long long* hdr, uint64_t cap) {
  const uint64_t n = hdr[0];
  return n < cap ? n : cap;
}

__global__ void __launch_bounds__(256) k_jr_count(const unsigned long long* __restrict__ rec,
                                                 const unsigned long long* hdr, uint64_t cap, uint32_t nb,
                                                 uint64_t nt, uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t h[];
  const uint64_t n = n_records(hdr, cap);
  const uint64_t t = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < nb; i += 256) h[i] = 0u;
  __syncthreads();
  const uint64_t a = t * kTile1, e = a + kTile1 < n ? a + kTile1 : n;
  for (uint64_t k = a + threadIdx.x; k < e; k += 8 * 256) {
    unsigned long long r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint64_t kk = k + (uint64_t)q * 256;
      r[q] = kk < e ? rec[kk] : ~0ull;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (r[q] != ~0ull) atomicAdd(&h[bucket_of(r[q], nb)], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nb; i += 256) counts[(uint64_t)i * nt + t] = h[i];
}

// exclusive scan of v[0, n) in place: block sums, their scan, then each block
// rescans its range from its base
__global__ void __launch_bounds__(256) k_scan_sums(const uint32_t* __restrict__ v, uint64_t n,
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

__global__ void __launch_bounds__(256) k_scan_apply(uint32_t* __restrict__ v, uint64_t n,
                                                   const unsigned long long* __restrict__ bsum) {
  __shared__ uint32_t s[256];
  const uint64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
  const uint64_t a = blockIdx.x * chunk, e = a + chunk < n ? a + chunk : n;
  uint32_t carry = (uint32_t)bsum[blockIdx.x];
  for (uint64_t k0 = a; k0 < e; k0 += 256) {
    const uint64_t k = k0 + threadIdx.x;
    const uint32_t x = k < e ? v[k] : 0u;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {      // inclusive scan (Hillis-Steele)
      const uint32_t y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
      __syncthreads();
      s[threadIdx.x] += y;
      __syncthreads();
    }
    if (k < e) v[k] = carry + s[threadIdx.x] - x;
    const uint32_t tot = s[255];
    __syncthreads();
    carry += tot;
  }
}

// Block-wide exclusive scan of v[0, n) in LDS with NT threads; returns the
// total.  part: LDS scratch of NT words.
template <int NT>
__device__ uint32_t block_exclusive_scan(uint32_t* v, uint32_t n, uint32_t* part) {
  const uint32_t per = (n + NT - 1) / NT, a = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t i = a; i < a + per && i < n; ++i) loc += v[i];
  part[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const uint32_t y = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - loc;
  for (uint32_t i = a; i < a + per && i < n; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  const uint32_t total = part[NT - 1];
  __syncthreads();
  return total;
}

// Per tile, sub-tiles of `sub` records are sorted by bucket in LDS and then
// written as contiguous runs to their buckets' ranges (consecutive threads,
// consecutive addresses).
template <int NT>
__global__ void __launch_bounds__(NT) k_jr_scatter(const unsigned long long* __restrict__ recA,
                                                    const unsigned long long* hdr, uint64_t cap, uint32_t nb,
                                                    uint64_t nt, const uint32_t* __restrict__ offs,
                                                    unsigned long long* __restrict__ recB, uint32_t sub) {
  extern __shared__ unsigned long long smem64[];
  unsigned long long* srt = smem64;                                   // [sub] records by bucket
  uint32_t* run = reinterpret_cast<uint32_t*>(smem64 + sub);          // [nb] next position per bucket
  uint32_t* pre = run + nb;                                           // [nb] counts, then prefix
  __shared__ uint32_t part[NT];
  const uint64_t n = n_records(hdr, cap);
  const uint64_t t = blockIdx.x;
  const uint64_t a = t * kTile1;
  if (a >= n) return;
  const uint64_t e = a + kTile1 < n ? a + kTile1 : n;
  for (uint32_t i = threadIdx.x; i < nb; i += NT) {
    run[i] = offs[(uint64_t)i * nt + t];
    pre[i] = 0u;
  }
  __syncthreads();
  constexpr int kMaxPer = 16;                                         // sub <= 16 NT
  for (uint64_t s0 = a; s0 < e; s0 += sub) {
    const uint32_t m = (uint32_t)(e - s0 < sub ? e - s0 : sub);
    unsigned long long r[kMaxPer];
    uint32_t bk[kMaxPer], rk[kMaxPer];
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      if (k < m) {
        r[q] = recA[s0 + k];
        bk[q] = bucket_of(r[q], nb);
        rk[q] = atomicAdd(&pre[bk[q]], 1u);
      }
    }
    __syncthreads();
    block_exclusive_scan<NT>(pre, nb, part);
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const uint32_t k = (uint32_t)q * NT + threadIdx.x;
      if (k < m) srt[pre[bk[q]] + rk[q]] = r[q];
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += NT) {
      const unsigned long long x = srt[k];
      const uint32_t b = bucket_of(x, nb);
      const uint64_t dst = (uint64_t)run[b] + (k - pre[b]);
      if (dst < n) recB[dst] = x;
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

// bucket b's records: [offs[b nt], offs[(b+1) nt]) (the last ends at n);
// parts[b] = exclusive prefix of ceil(len_b / kPart) over buckets
__global__ void __launch_bounds__(1024) k_jr_items(const uint32_t* __restrict__ offs,
                                                  unsigned long long* hdr, uint64_t cap, uint32_t nb,
                                                  uint64_t nt, uint32_t* __restrict__ parts) {
  __shared__ uint32_t s[1024];
  const uint64_t n = n_records(hdr, cap);
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t loc = 0;
  for (uint32_t b = b0; b < b0 + per && b < nb; ++b) {
    const uint64_t lo = offs[(uint64_t)b * nt];
    const uint64_t hi = b + 1 < nb ? offs[(uint64_t)(b + 1) * nt] : n;
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
    const uint64_t lo = offs[(uint64_t)b * nt];
    const uint64_t hi = b + 1 < nb ? offs[(uint64_t)(b + 1) * nt] : n;
    run += (uint32_t)((hi - lo + kPart - 1) / kPart);
  }
  if (threadIdx.x == 1023) {
    parts[nb] = s[1023];
    hdr[1] = 0ull;
  }
}

__global__ void __launch_bounds__(1024) k_jr_sum(const unsigned long long* __restrict__ recB,
                                                unsigned long long* hdr, uint64_t cap, uint32_t nb, uint64_t nt,
                                                const uint32_t* __restrict__ offs,
                                                const uint32_t* __restrict__ parts, uint64_t n_slots,
                                                unsigned long long* __restrict__ jq) {
  extern __shared__ uint32_t acc[];
  __shared__ uint32_t s_item;
  const uint64_t n = n_records(hdr, cap);
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
    const uint64_t start = offs[(uint64_t)b * nt];
    const uint64_t end = b + 1 < nb ? offs[(uint64_t)(b + 1) * nt] : n;
    const uint64_t r0 = start + (uint64_t)(item - parts[b]) * kPart;
    const uint64_t r1 = r0 + kPart < end ? r0 + kPart : end;
    const bool shared_bucket = parts[b + 1] - parts[b] > 1;
    const uint64_t base = (uint64_t)b * kBucketSlots;
    for (uint32_t i = threadIdx.x; i < kBucketSlots; i += 1024) acc[i] = 0u;
    __syncthreads();
    for (uint64_t k = r0 + threadIdx.x; k < r1; k += 8 * 1024) {
      unsigned long long r[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint64_t kk = k + (uint64_t)q * 1024;
        r[q] = kk < r1 ? recB[kk] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint64_t slot = r[q] >> kRecValBits;
        const uint32_t val = (uint32_t)(r[q] & kValMask);
        const uint64_t i = slot - base;
        if (val != 0u && i < kBucketSlots) {
          const uint32_t old = atomicAdd(&acc[i], val);
          if (old + val < old) atomicAdd(&jq[slot], 1ull << 32);
        }
      }
    }
    __threadfence();
    __syncthreads();
    const uint64_t ns = n_slots - base < kBucketSlots ? n_slots - base : kBucketSlots;
    for (uint32_t i = threadIdx.x; i < ns; i += 1024) {
      const uint32_t v = acc[i];
      if (v) {
        if (shared_bucket) atomicAdd(&jq[base + i], (unsigned long long)v);
        else jq[base + i] += v;
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
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += (bytes + 255) & ~255ull;
    return o;
  };
  J.hdr = take(64);
  J.counts = take(4 * J.n_buckets * J.n_tiles);
  J.prefix = take(8 * (kScanBlocks + 1));
  J.parts = take(4 * (J.n_buckets + 1));
  J.recA = take(8 * capacity);
  J.recB = take(8 * capacity);
  J.total = off;
  return J;
}

hipError_t launch_jrec_accumulate(mcrt_ctx* c, const mcrt_run_opts& o, uint64_t* jq, hipStream_t s) {
  const uint64_t n_slots = (uint64_t)c->d.n_lambda * (uint64_t)c->d.n_cells;
  const JrecLayout J = jrec_layout(n_slots, o.jrec_capacity);
  unsigned char* ws = static_cast<unsigned char*>(o.jrec_ws);
  auto* hdr = reinterpret_cast<unsigned long long*>(ws + J.hdr);
  auto* counts = reinterpret_cast<uint32_t*>(ws + J.counts);
  auto* bsum = reinterpret_cast<unsigned long long*>(ws + J.prefix);
  auto* parts = reinterpret_cast<uint32_t*>(ws + J.parts);
  auto* recA = reinterpret_cast<unsigned long long*>(ws + J.recA);
  auto* recB = reinterpret_cast<unsigned long long*>(ws + J.recB);
  auto* tally = reinterpret_cast<unsigned long long*>(jq);
  const uint32_t nb = (uint32_t)J.n_buckets;
  const uint64_t nt = J.n_tiles, cap = J.capacity, nc = (uint64_t)nb * nt;
  k_jr_count<<<(unsigned)nt, 256, 4 * (size_t)nb, s>>>(recA, hdr, cap, nb, nt, counts);
  k_scan_sums<<<kScanBlocks, 256, 0, s>>>(counts, nc, bsum);
  k_scan_top<<<1, 64, 0, s>>>(bsum);
  k_scan_apply<<<kScanBlocks, 256, 0, s>>>(counts, nc, bsum);
  // few buckets: 512-thread blocks on 8192-record sub-tiles, two per CU, so
  // one block's loads overlap the other's sort; otherwise one 1024-thread
  // block per CU with the largest power-of-two sub-tile (<= 16384 records)
  // whose sort buffer fits beside the two bucket arrays in 160 KB of LDS
  if (8 * (size_t)nb <= 12 * 1024) {
    const uint32_t sub = 8192;
    k_jr_scatter<512><<<(unsigned)nt, 512, (size_t)sub * 8 + 8 * (size_t)nb, s>>>(recA, hdr, cap, nb, nt,
                                                                                 counts, recB, sub);
  } else {
    uint32_t sub = 16384;
    while (sub > 1024 && (size_t)sub * 8 + 8 * (size_t)nb + 4096 + 256 > 160 * 1024) sub >>= 1;
    k_jr_scatter<1024><<<(unsigned)nt, 1024, (size_t)sub * 8 + 8 * (size_t)nb, s>>>(recA, hdr, cap, nb, nt,
                                                                                   counts, recB, sub);
  }
  k_jr_items<<<1, 1024, 0, s>>>(counts, hdr, cap, nb, nt, parts);
  k_jr_sum<<<(unsigned)c->n_cu, 1024, 4 * kBucketSlots, s>>>(recB, hdr, cap, nb, nt, counts, parts, n_slots, tally);
  return hipGetLastError();
}

}  // namespace mcrt

extern "C" int32_t mcrt_jrec_ws_bytes(const mcrt_ctx* ctx, uint64_t capacity, uint64_t* bytes) {
  if (!ctx || !bytes) return MCRT_E_INVALID;
  const uint64_t n_slots = (uint64_t)ctx->d.n_lambda * (uint64_t)ctx->d.n_cells;
  if (capacity < mcrt::kRecChunk || capacity > (1ull << 31)) return MCRT_E_INVALID;
  if (ctx->d.max_level > 7 || n_slots >= (1ull << 40)) return MCRT_E_UNSUPPORTED;
  const mcrt::JrecLayout J = mcrt::jrec_layout(n_slots, capacity);
  if (J.n_buckets > (uint64_t)mcrt::kMaxBuckets || J.n_buckets * J.n_tiles > (1ull << 26))
    return MCRT_E_UNSUPPORTED;
  *bytes = J.total;
  return MCRT_OK;
}
