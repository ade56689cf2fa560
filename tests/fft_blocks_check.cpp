// Host build of the small-DFT building blocks of the FFT passes (fft_core.h):
// prints, for every supported radix, the length-R DFT of a fixed input in
// both directions (natural order), and the same for the upper-half-zero DFT
// of the even radices, as "R dir kind k re im" lines for a checker to compare
// with a reference DFT.
#include <cmath>
#include <cstdio>

#include "fft_core.h"

using namespace aim::fftc;

template <int R, bool INV, bool UZ>
void emit() {
  double2 v[R];
  for (int i = 0; i < R; ++i) {
    v[i].x = std::sin(1.3 * i + 0.2);
    v[i].y = std::cos(0.7 * i * i);
    if (UZ && i >= R / 2) {  // must not be read
      v[i].x = NAN;
      v[i].y = NAN;
    }
  }
  if constexpr (UZ) dft_upper_zero<R, INV, double2>(v);
  else Dft<R, INV, double2>::run(v);
  for (int k = 0; k < R; ++k)
    std::printf("%d %d %d %d %.17g %.17g\n", R, INV ? 1 : 0, UZ ? 1 : 0, k, v[k].x, v[k].y);
}

int main() {
#define AIM_EMIT(R)                                   \
  emit<R, false, false>();                            \
  emit<R, true, false>();                             \
  if constexpr (R % 2 == 0) {                         \
    emit<R, false, true>();                           \
    emit<R, true, true>();                            \
  }
  AIM_FOR_EACH_RADIX(AIM_EMIT)
#undef AIM_EMIT
  return 0;
}
