// Host-side known-answer generator for Philox4x32-10 using rocRAND's
// independent engine.  Reads lines "c0 c1 c2 c3 k0 k1" (hex, 32-bit words)
// on stdin and prints the four output words of ten rounds applied to that
// counter under that key.  The engine's (subsequence, offset) arguments map
// to the counter as (offset/4) -> (c0, c1) and subsequence -> (c2, c3).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (static_cast<unsigned long long>(k1) << 32) | k0;
    unsigned long long sub = (static_cast<unsigned long long>(c3) << 32) | c2;
    unsigned long long blk = (static_cast<unsigned long long>(c1) << 32) | c0;
    rocrand_device::philox4x32_10_engine e(seed, sub, 4ULL * blk);
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
