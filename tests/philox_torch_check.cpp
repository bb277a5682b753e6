// Third-source check of Philox4x32-10 words: PyTorch's header-only CPU engine
// (ATen/core/PhiloxRNGEngine.h), built on the host by the oracle tests.
//
// The engine's state is a counter (offset_lo, offset_hi, subsequence_lo,
// subsequence_hi) and a key (seed_lo, seed_hi); the first four words it returns are
// the Philox block of that counter under that key.  Reads lines "c0 c1 c2 c3 k0 k1"
// (decimal) from stdin and prints the four words of each block in decimal.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c[4], k[2];
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    const uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
    const uint64_t subsequence = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
    const uint64_t offset = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    at::philox_engine eng(seed, subsequence, offset);
    const uint32_t w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
