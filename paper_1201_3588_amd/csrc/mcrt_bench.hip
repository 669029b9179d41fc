// Random-access microbenchmark: the achievable rate of the transaction mix of
// the transport kernel (uniformly random 64-bit atomic adds over a tally of the
// path-length tally's size, random 4-byte loads over the density grid), used
// as the ceiling against which the traversal kernel is measured.
#include "mcrt_internal.h"

namespace {

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  // splitmix64 finaliser (Steele, Lea & Flood 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_rand_atomics(unsigned long long* __restrict__ t,
                                                      unsigned long long n_slots,
                                                      unsigned long long ops_per_thread,
                                                      unsigned long long seed) {
  const unsigned long long tid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long s = mix64(seed ^ (tid * 0x9E3779B97F4A7C15ull));
  for (unsigned long long i = 0; i < ops_per_thread; ++i) {
    s = mix64(s + 0x9E3779B97F4A7C15ull);
    atomicAdd(&t[s % n_slots], 1ull);
  }
}

__global__ void __launch_bounds__(256) k_rand_loads(const float* __restrict__ t,
                                                    unsigned long long n_load,
                                                    unsigned long long ops_per_thread,
                                                    unsigned long long seed, float* sink) {
  const unsigned long long tid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long s = mix64(seed ^ (tid * 0x9E3779B97F4A7C15ull));
  float acc = 0.0f;
  // a power-of-two size takes a mask instead of the 64-bit remainder, whose
  // emulation would make the loop bound by arithmetic rather than by memory
  const unsigned long long mask = (n_load & (n_load - 1)) == 0 ? n_load - 1 : 0;
  for (unsigned long long i = 0; i < ops_per_thread; ++i) {
    s = mix64(s + 0x9E3779B97F4A7C15ull);
    acc += t[mask ? (s & mask) : s % n_load];
  }
  if (acc == -1.0f) sink[0] = acc;   // keeps the loads alive
}

}  // namespace

extern "C" int32_t mcrt_bench_random(uint64_t* table, uint64_t n_slots, const float* loads,
                                     uint64_t n_load, uint64_t n_ops, uint64_t seed, int32_t mode,
                                     float* sink, hipStream_t stream) {
  if (n_ops == 0) return MCRT_OK;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned blocks = (unsigned)ncu * 16;
  const unsigned long long threads = (unsigned long long)blocks * 256;
  const unsigned long long per = (n_ops + threads - 1) / threads;
  if (mode == 0) {
    if (!table || n_slots == 0) return MCRT_E_INVALID;
    k_rand_atomics<<<blocks, 256, 0, stream>>>(reinterpret_cast<unsigned long long*>(table), n_slots,
                                               per, seed);
  } else if (mode == 1) {
    if (!loads || n_load == 0 || !sink) return MCRT_E_INVALID;
    k_rand_loads<<<blocks, 256, 0, stream>>>(loads, n_load, per, seed, sink);
  } else {
    return MCRT_E_INVALID;
  }
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}
