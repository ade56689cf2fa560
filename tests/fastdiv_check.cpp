// Host check of the multiply-high division of the x pass's work numbering
// (fast_div in fft_map.h) against plain integer division: every divisor up
// to 4096, powers of two and their neighbours, and pseudo-random divisors up
// to 2^31 - 1, each with numerators at the edges (0, multiples of d and their
// neighbours, 2^31 - 1) and pseudo-random ones below 2^31. Prints
// "checked <count> mismatches <count>".
#include <cstdint>
#include <cstdio>
#include <vector>

#include "fft_map.h"

using namespace aim::fftk;

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint32_t next31() {  // splitmix64, top 31 bits
  uint64_t z = (state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (uint32_t)(z >> 33);
}

int main() {
  std::vector<uint32_t> ds;
  for (uint32_t d = 1; d <= 4096; ++d) ds.push_back(d);
  for (int k = 12; k < 31; ++k)
    for (int64_t e = -1; e <= 1; ++e) ds.push_back((uint32_t)((1ll << k) + e));
  ds.push_back(0x7fffffffu);
  for (int i = 0; i < 2000; ++i) {
    const uint32_t d = next31();
    if (d) ds.push_back(d);
  }
  uint64_t checked = 0, bad = 0;
  for (uint32_t d : ds) {
    const FastDiv f = make_fastdiv(d);
    auto check = [&](int64_t n) {
      if (n < 0 || n > 0x7fffffffll) return;
      ++checked;
      if (fast_div((uint32_t)n, f) != (uint32_t)n / d) ++bad;
    };
    check(0);
    check(0x7fffffffll);
    for (int64_t q : {(int64_t)1, (int64_t)2, (int64_t)3, (int64_t)7, (int64_t)1000,
                      (int64_t)(0x7fffffffll / d)}) {
      check(q * d - 1);
      check(q * d);
      check(q * d + 1);
    }
    for (int i = 0; i < 200; ++i) check(next31());
  }
  std::printf("checked %llu mismatches %llu\n", (unsigned long long)checked,
              (unsigned long long)bad);
  return 0;
}
