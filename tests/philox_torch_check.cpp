// Cross-check for the oracle's Philox-4x32-10: an independent implementation,
// PyTorch's at::philox_engine (ATen/core/PhiloxRNGEngine.h), evaluated on the
// counters/keys read from stdin.  Input lines: c0 c1 c2 c3 k0 k1 (decimal).
// The engine's counter is (offset_lo, offset_hi, subsequence_lo,
// subsequence_hi) and its key is the seed, so one block is reproduced by
// philox_engine(seed = k0 | k1<<32, subsequence = c2 | c3<<32,
// offset = c0 | c1<<32) followed by four calls.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c[4], k[2];
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    uint64_t seed = k[0] | (k[1] << 32);
    uint64_t subseq = c[2] | (c[3] << 32);
    uint64_t offset = c[0] | (c[1] << 32);
    at::philox_engine eng(seed, subseq, offset);
    uint32_t a = eng(), b = eng(), d = eng(), e = eng();
    std::printf("%u %u %u %u\n", a, b, d, e);
  }
  return 0;
}
