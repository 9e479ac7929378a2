// Host-only driver around rocRAND's Philox4x32-10 engine, used by the test
// suite as an external known-answer source for the oracle's generator.
// Reads lines "seed step inst" and prints the four output words of the block
// at counter (step, inst, 0, 0) under key (lo32(seed), hi32(seed)).  The
// engine starts at counter 0 and advances by `offset` 32-bit outputs, i.e.
// offset / 4 blocks carried into counter words 0 and 1.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned long long seed, step, inst;
  while (std::scanf("%llu %llu %llu", &seed, &step, &inst) == 3) {
    const unsigned long long block = (inst << 32) | step;
    rocrand_device::philox4x32_10_engine e(seed, 0ull, 4ull * block);
    const uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
