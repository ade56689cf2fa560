// FFT pass dispatch for double2: the run-time length selects the compiled kernel set.
#include "fft_kernels.h"

namespace aim {
void fft_pass_strided(const double2 *in, double2 *out, const FftPlan &pl, int n_in, int n_out,
                      int64_t outer, int64_t inner, const fftk::LineMap &imap,
                      const fftk::LineMap &omap, bool inverse, const double2 *tw, int row_bytes,
                      hipStream_t s) {
  if (outer <= 0 || inner <= 0) return;
  switch (pl.P) {
#define AIM_X(P, a, b, c)                                                                      \
  case P:                                                                                      \
    fftk::launch_strided<double, fftk::PlanC<a, b, c>>(in, out, n_in, n_out, outer, inner,         \
                                                    imap, omap, inverse, tw, row_bytes, s);               \
    return;
    AIM_FOR_EACH_FFT_PLAN(AIM_X)
#undef AIM_X
    default:
      break;
  }
  fftk::bad_length(pl.P);
}
}  // namespace aim
