// Third-party cross-check of the oracle's Philox4x32-10: reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four output words of rocRAND's
// philox4x32_10 engine positioned at counter (c0, c1, c2, c3) under key
// (k0, k1).  Host-only; used by tests/test_oracle_philox.py.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long key = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(key, subseq, offset);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
