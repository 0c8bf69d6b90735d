// Host-side check program: evaluates rocRAND's Philox4x32-10 routine on
// counter/key tuples read from stdin ("c0 c1 c2 c3 k0 k1" in hex, one per line)
// and prints the four output words in hex.  Used by the CPU test suite to pin
// the oracle's Philox against an independent library implementation.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct PhiloxProbe : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  PhiloxProbe e;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 c;
    c.x = c0; c.y = c1; c.z = c2; c.w = c3;
    uint2 k;
    k.x = k0; k.y = k1;
    uint4 r = e.ten_rounds(c, k);
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
