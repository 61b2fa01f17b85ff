// Prints rocRAND philox4x32_10 first outputs for (seed, subsequence) pairs read
// from stdin, evaluated on the host.  Used by the oracle's RNG pin: rocRAND's
// engine evaluates Philox4x32-10 at counter (0, 0, subsequence) with key = seed.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned long long seed, subseq;
  while (std::scanf("%llx %llx", &seed, &subseq) == 2) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, 0, &st);
    uint4 v = rocrand4(&st);
    std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
