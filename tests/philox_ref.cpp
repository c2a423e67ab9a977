// Reference Philox4x32-10 outputs from PyTorch's ATen engine (an implementation
// independent of the oracle's).  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on
// stdin and prints the four output words.  ATen packs its engine state as
// counter = {lo(offset), hi(offset), lo(subsequence), hi(subsequence)} and
// key = {lo(seed), hi(seed)}; the first four calls return words 0..3.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = k0 | (k1 << 32), sub = c2 | (c3 << 32), off = c0 | (c1 << 32);
    at::philox_engine e(seed, sub, off);
    uint32_t a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
