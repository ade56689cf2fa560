// FFT pass dispatch for double2: the run-time length selects the compiled kernel set.
#include "fft_kernels.h"

namespace aim {
void fft_mid_pass(double2 *data, const FftPlan &pl, int n_x, int nfield, int Py, int Pz, int Hx,
                  int Hy, int Hz, const double2 *ghat, const double2 *tw, int blk, int64_t fstride,
                  int row_bytes, hipStream_t s) {
  (void)Hx;
  if (nfield <= 0) return;
  switch (pl.P) {
#define AIM_X(P, a, b, c)                                                                   \
  case P:                                                                                   \
    fftk::launch_mid<double, fftk::PlanC<a, b, c>>(data, n_x, nfield, Py, Pz, Hy, Hz, ghat, tw, \
                                                blk, fstride, row_bytes, s);                           \
    return;
    AIM_FOR_EACH_FFT_PLAN(AIM_X)
#undef AIM_X
    default:
      break;
  }
  fftk::bad_length(pl.P);
}
}  // namespace aim
