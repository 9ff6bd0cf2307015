// Known-answer probe: Philox-4x32-10 as implemented by rocRAND
// (rocrand/rocrand_philox4x32_10.h), compiled for the host. Reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four 32-bit outputs.
// Mapping: seed -> key (lo, hi); subsequence -> counter words 2, 3;
// offset counts 32-bit outputs, so 4*(c0 | c1<<32) -> counter words 0, 1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32), subseq = c2 | (c3 << 32);
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
