// Internal declarations shared by the HIP translation units of libmcrt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "mcrt.h"

namespace mcrt {

constexpr double kC = 2.99792458e10;     // cm s^-1
constexpr double kH = 6.62607015e-27;    // erg s
constexpr double kKB = 1.380649e-16;     // erg K^-1
constexpr double kPi = 3.14159265358979323846;

// Philox4x32-10 (Salmon et al. 2011): round multipliers and key increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// (0,1] uniform from the top 24 bits of a word (exact in FP32 and FP64).
__device__ __forceinline__ double u24(uint32_t w) {
  return (double)((w >> 8) + 1u) * (1.0 / 16777216.0);
}

__device__ __forceinline__ double planck_nu(double nu, double T) {
  const double x = kH * nu / (kKB * T);
  return 2.0 * kH * nu * nu * nu / (kC * kC) / expm1(x);
}

// first index j in [0,n) with cdf[j] >= u; cdf[n-1] == 1
__device__ __forceinline__ int cdf_search(const double* __restrict__ cdf, int n, double u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cdf[mid] >= u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

struct Layout {
  uint64_t nu, dnu, src_cdf, kext, albedo, gpar, sp_cdf, Tk, E, R, Bt, Wt, xk;
  uint64_t kext32, g32, rho_h32, level, leaf_lo, binfo, pah_slot, scratch, total;
};

// run scratch inside the tables buffer (zeroed by a fill kernel per run)
struct RunScratch {
  unsigned long long work_counter;
  unsigned long long bad_input;
  unsigned long long peel_count;     // next-event records claimed by the run
  unsigned long long pad[29];
};

Layout make_layout(const mcrt_desc& d);

// The packed base-cube table (entry + FP32 density term) of the FP32
// transport is stored in bricks of 4 x 2 x 2 base cubes, one 128-byte cache
// line each: a packet stepping to a neighbour in y or z then stays in the
// line half of the time (in raster order never), in x three times in four.
// Bricks are in raster order over ceil(nb/4) x ceil(nb/2) x ceil(nb/2).
// (32-bit arithmetic: nb^3 <= 2^31 keeps every index below 2^32.)
__host__ __device__ __forceinline__ uint32_t binfo_index(int nb, int bx, int by, int bz) {
  const uint32_t nx4 = (uint32_t)(nb + 3) >> 2, ny2 = (uint32_t)(nb + 1) >> 1;
  const uint32_t brick = ((uint32_t)(bz >> 1) * ny2 + (uint32_t)(by >> 1)) * nx4 + (uint32_t)(bx >> 2);
  return brick * 16u + (uint32_t)(((bz & 1) << 3) | ((by & 1) << 2) | (bx & 3));
}
__host__ __device__ __forceinline__ uint64_t binfo_entries(int nb) {
  return (uint64_t)((nb + 3) >> 2) * (uint64_t)((nb + 1) >> 1) * (uint64_t)((nb + 1) >> 1) * 16;
}

// Deferred path-length tally: the transport appends one 64-bit record per
// path segment, (tally index << 24) | fixed-point length, in chunks of
// kRecChunk claimed per wave; a partition by tally range and an LDS sum then
// add them to the tally (mcrt_jdefer.hip).
constexpr uint64_t kRecChunk = 4096;
constexpr int kRecValBits = 24;
constexpr uint64_t kBucketSlots = 40704;        // tally words per LDS bucket (u32 partial sums)
constexpr uint64_t kTile1 = 1ull << 18;         // records per partition tile
constexpr uint64_t kOneLevelMax = 1536;         // more buckets: two partition levels
constexpr uint64_t kMaxBuckets = 1ull << 20;
constexpr uint64_t kMaxRecords = 1ull << 35;     // workspace capacity limit (64-bit offsets)
struct JrecLayout {
  uint64_t n_buckets, n_tiles, capacity;
  bool two_level;
  uint64_t fpc, nc;                               // two levels: buckets per coarse range, coarse ranges
  uint64_t hdr, tb, parts, lvl1, lvl2, recA, recB, total;   // byte offsets
};
JrecLayout jrec_layout(uint64_t n_slots, uint64_t capacity);
// The last deferred-tally range a context ran: its workspace, capacity,
// seed, pass size, the packet id after it and how many consecutive ranges
// led up to it.  A range that continues it sizes its partition regions from
// the record totals of the ranges before.
struct JrecChain {
  const void* ws = nullptr;
  uint64_t capacity = 0, seed = 0, n_total = 0, next_id = 0, length = 0;
};

}  // namespace mcrt

namespace mcrt {
// observers of the escape images, as the kernel uses them: unit line of sight
// n, plane axes e1, e2, and the grid origin relative to the image centre (cm)
struct ImgP {
  int n_obs, npix, n_l;
  int lsel[MCRT_MAX_IMAGE_BINS];
  double n[MCRT_MAX_OBSERVERS][3], e1[MCRT_MAX_OBSERVERS][3], e2[MCRT_MAX_OBSERVERS][3];
  double off[3], h, w, cos_cone;
  unsigned long long* image;
};
}  // namespace mcrt

struct mcrt_ctx {
  mcrt_desc d;
  mcrt::ImgP img{};
  mcrt::Layout lay;
  int n_pah = 0;
  bool tables_built = false;
  unsigned char* tables = nullptr;   // caller-owned device buffer
  mcrt_source src{};
  std::string err;
  int device = 0;
  int n_cu = 256;
  mcrt::JrecChain jchain;
};

namespace mcrt {
hipError_t launch_checks(mcrt_ctx* c, hipStream_t s);
hipError_t launch_build_tables(mcrt_ctx* c, hipStream_t s);
hipError_t launch_transport(mcrt_ctx* c, uint64_t first_id, uint64_t n, const mcrt_run_opts& o,
                            const mcrt_tallies& t, hipStream_t s);
hipError_t launch_jrec_accumulate(mcrt_ctx* c, const mcrt_run_opts& o, uint64_t first_id, uint64_t n_packets,
                                  uint64_t* jq, hipStream_t s);
hipError_t launch_temperatures(mcrt_ctx* c, const uint64_t* nabs, uint64_t n_total, double* T,
                               hipStream_t s);
hipError_t launch_thin_field(mcrt_ctx* c, float* J, hipStream_t s);
hipError_t launch_cell_mass(mcrt_ctx* c, double* mass, hipStream_t s);
hipError_t launch_mean_intensity(mcrt_ctx* c, const uint64_t* jq, uint64_t n_total, float* J,
                                 hipStream_t s);
}  // namespace mcrt
