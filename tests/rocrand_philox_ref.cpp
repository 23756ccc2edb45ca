// Independent Philox4x32-10 reference for the oracle's pin: ROCm's rocRAND
// engine, host side.  Reads "c0 c1 c2 c3 k0 k1" lines, prints the 4 output words.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
