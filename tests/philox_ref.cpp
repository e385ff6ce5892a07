// Test helper: prints Philox4x32-10 output blocks computed by rocRAND's host
// implementation, an implementation independent of both the oracle and the HIP
// library.  stdin: "k0 k1" then lines "c0 c1 c2 c3" (decimal); stdout: one
// line of four hex words per counter.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// Exposes the engine's ten-round bijection on an explicit counter and key.
struct Probe : rocrand_device::philox4x32_10_engine {
  static uint4 block(uint4 c, uint2 k) {
    Probe p;
    return p.ten_rounds(c, k);
  }
};

int main() {
  unsigned long long k0, k1, c0, c1, c2, c3;
  if (std::scanf("%llu %llu", &k0, &k1) != 2) return 1;
  const uint2 key = {(unsigned int)k0, (unsigned int)k1};
  while (std::scanf("%llu %llu %llu %llu", &c0, &c1, &c2, &c3) == 4) {
    const uint4 c = {(unsigned int)c0, (unsigned int)c1, (unsigned int)c2, (unsigned int)c3};
    const uint4 v = Probe::block(c, key);
    std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
