// Prints rocRAND's philox4x32_10 block for counter (pid_lo, pid_hi, e, k) and
// key (seed_lo, seed_hi): rocrand_init places the subsequence in counter words
// 2..3 and offset/4 in words 0..1.  Host-side use of the header-only engine.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc % 4 != 1) return 2;
  for (int a = 1; a < argc; a += 4) {
    unsigned long long seed = std::strtoull(argv[a], nullptr, 0);
    unsigned long long pid = std::strtoull(argv[a + 1], nullptr, 0);
    unsigned long long e = std::strtoull(argv[a + 2], nullptr, 0);
    unsigned long long k = std::strtoull(argv[a + 3], nullptr, 0);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, e | (k << 32), 4ull * pid, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
