// Pipelined y / x / y passes for double2: the run-time length selects the
// compiled kernel (lengths >= 64 with two or three stages).
#include "fft_kernels.h"

namespace aim {
namespace {
template <int a, int b, int c>
void xy_dispatch(const double2 *gz, double2 *g2, double2 *g1, int Nx, int Ny, int F, int G, int Py, int Pz,
                 int Hy, int Hz, const double2 *ghat, const double2 *twx, const double2 *twy, int blk,
                 int64_t V2, const fftk::LineMap &m1y, const fftk::LineMap &m2, hipStream_t s) {
  if constexpr (a * b * c >= 64)
    fftk::launch_xy<double, fftk::PlanC<a, b, c>>(gz, g2, g1, Nx, Ny, F, G, Py, Pz, Hy, Hz, ghat, twx,
                                             twy, blk, V2, m1y, m2, s);
  else
    fftk::bad_length(a * b * c);
}
}  // namespace

void fft_xy_pipeline(const double2 *gz, double2 *g2, double2 *g1, const FftPlan &pl, int Nx, int Ny,
                     int F, int G, int Py, int Pz, int Hy, int Hz, const double2 *ghat,
                     const double2 *twx, const double2 *twy, int blk, int64_t V2,
                     const fftk::LineMap &m1y, const fftk::LineMap &m2, hipStream_t s) {
  switch (pl.P) {
#define AIM_X(P, a, b, c)                                                                       \
  case P:                                                                                       \
    xy_dispatch<a, b, c>(gz, g2, g1, Nx, Ny, F, G, Py, Pz, Hy, Hz, ghat, twx, twy, blk, V2, m1y, \
                         m2, s);                                                                \
    return;
    AIM_FOR_EACH_FFT_PLAN(AIM_X)
#undef AIM_X
    default:
      break;
  }
  fftk::bad_length(pl.P);
}

}  // namespace aim
