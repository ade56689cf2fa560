// Anterpolation fused with the forward z pass, double arithmetic: the run-time
// FFT length selects the compiled kernel.
#include "fft_anterp.h"

namespace aim {
bool anterp_fftz(const double2 *x, int64_t ldx, int nrhs, const int32_t *node_ptr,
                 const int32_t *ent_col, const double *lamT, int Nz, int64_t nlines, double2 *out,
                 int64_t out_ls, int64_t out_fstride, const double2 *tw, const FftPlan &pl,
                 hipStream_t s) {
  switch (pl.P) {
#define AIM_X(P, a, b, c)                                                                   \
  case P:                                                                                   \
    return fftk::launch_anterp_fftz<double, double, fftk::PlanC<a, b, c>>(x, ldx, nrhs, node_ptr, ent_col, \
                                                            lamT, Nz, nlines, out, out_ls,   \
                                                            out_fstride, tw, s);
    AIM_FOR_EACH_FFT_PLAN(AIM_X)
#undef AIM_X
    default:
      break;
  }
  fftk::bad_length(pl.P);
  return false;
}

}  // namespace aim
