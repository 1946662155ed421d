// Prints Philox4x32-10 outputs computed by rocRAND's host-callable engine.
//
// Test infrastructure: an independent implementation of the published
// Philox4x32-10 (Salmon et al., SC'11) used to pin the oracle's generator.
// Input lines on stdin: "c0 c1 c2 c3 k0 k1" (decimal); output lines: the four
// 32-bit output words of that counter/key.
//
// rocRAND's engine starts from counter (0,0,0,0) with key = seed; skipping
// `subsequence` adds to counter words (2,3) and skipping `offset` numbers adds
// offset/4 to counter words (0,1). With offset = 4*(c0 + 2^32 c1) and
// subsequence = c2 + 2^32 c3 the engine's first output block is
// Philox(c, k). The offset is a 64-bit count of numbers, so counter word 1
// must stay below 2^30.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const unsigned long long seed = k0 | (k1 << 32);
    const unsigned long long sub = c2 | (c3 << 32);
    const unsigned long long off = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned w0 = e.next(), w1 = e.next(), w2 = e.next(), w3 = e.next();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
