// Test helper: prints rocRAND's Philox4x32-10 block function for counter/key
// lines read from stdin ("c0 c1 c2 c3 k0 k1" per line). Used only by the
// oracle's tests to pin the oracle's own Philox against an independent
// implementation; the GPU library does not use it.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  probe p;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 c = {c0, c1, c2, c3};
    uint2 k = {k0, k1};
    uint4 r = p.block(c, k);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
