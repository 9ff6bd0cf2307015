// Known-answer probe: Philox-4x32-10 as implemented by PyTorch's
// at::Philox4_32 (ATen/core/PhiloxRNGEngine.h). Reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four 32-bit outputs.
// Mapping: seed -> key (lo, hi); subsequence -> counter words 2, 3;
// offset (in 128-bit groups) -> counter words 0, 1.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = k0 | (k1 << 32), subseq = c2 | (c3 << 32), offset = c0 | (c1 << 32);
    at::Philox4_32 eng(seed, subseq, offset);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
