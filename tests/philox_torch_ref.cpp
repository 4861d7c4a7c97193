// Reference Philox4x32-10 blocks from PyTorch's own engine (ATen/core/PhiloxRNGEngine.h), used by
// the tests as an independent implementation of the SC'11 generator.  Reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four output words of the block for that counter and key.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t subsequence = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::Philox4_32 engine(seed, subsequence, offset);
    uint32_t a = engine(), b = engine(), c = engine(), d = engine();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
