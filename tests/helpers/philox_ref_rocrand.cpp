// Test helper: Philox4x32-10 blocks from rocRAND's header-only engine, run on
// the host.  Same stdin/stdout format as philox_ref_aten.cpp.  rocRAND puts
// the subsequence in counter words 2-3 and offset/4 in words 0-1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (k1 << 32) | k0;
    unsigned long long subseq = (c3 << 32) | c2;
    unsigned long long block = (c1 << 32) | c0;
    rocrand_device::philox4x32_10_engine eng(seed, subseq, 0);
    eng.discard(block * 4ull);   // 4 outputs per counter value
    uint4 r = eng.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
