// Test helper: Philox4x32-10 blocks from PyTorch's header-only ATen engine.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin, prints the 4 output
// words.  ATen keys by the seed, puts the subsequence in counter words 2-3
// and the offset (in 128-bit blocks) in counter words 0-1.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (k1 << 32) | k0;
    uint64_t subseq = (c3 << 32) | c2;
    uint64_t offset = (c1 << 32) | c0;
    at::Philox4_32 eng(seed, subseq, offset);
    uint32_t x0 = eng(), x1 = eng(), x2 = eng(), x3 = eng();
    std::printf("%u %u %u %u\n", x0, x1, x2, x3);
  }
  return 0;
}
