// Bistatic radar cross section sigma_theta_theta (FP64).
//
// The paper measures accuracy through the VV bistatic RCS over the sphere of
// directions (Section 2.2, eq. 1). With J = sum_n I_n f_n, the radiation
// vector is N(r_hat) = int J exp(+j k r_hat . r') dS' and, for a unit incident
// field, sigma_tt = (k eta)^2 / (4 pi) |theta_hat . N|^2. The current is first
// collapsed onto the 7 quadrature points of every triangle (weights A w
// included); then each thread sums one direction over all points, which are
// staged through LDS.
#include <cmath>

#include "aim_internal.h"
#include "geom_device.h"

namespace aim {
using namespace geo;

namespace {

// per triangle quadrature point: position (3) and A w J (3 complex)
__global__ void k_point_currents(const int32_t *tris, const double *verts, const double *area,
                                 const int32_t *tri_basis, const double *len, const double2 *x,
                                 int64_t ldx, int nrhs, int64_t nt, double *pos, double2 *J) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt * 7) return;
  const int64_t tri = t / 7;
  const int p = (int)(t - tri * 7);
  D3 T[3];
  for (int c = 0; c < 3; ++c) T[c] = vtx(verts, tris[3 * tri + c]);
  double w;
  const D3 r = quad_point(T, p, &w);
  pos[3 * t] = r.x;
  pos[3 * t + 1] = r.y;
  pos[3 * t + 2] = r.z;
  const double A = area[tri];
  for (int rr = 0; rr < nrhs; ++rr) {
    double jr[3] = {0, 0, 0}, ji[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
      const int code = tri_basis[3 * tri + i];
      if (code < 0) continue;
      const int64_t n = code >> 1;
      const double s = (code & 1) ? -1.0 : 1.0;
      // f_n = s l / (2A) (r - v_i) on this triangle, v_i the free vertex
      const double c = s * len[n] / (2.0 * A) * A * w;
      const D3 d = r - T[i];
      const double2 I = x[(int64_t)rr * ldx + n];
      jr[0] += c * d.x * I.x;
      ji[0] += c * d.x * I.y;
      jr[1] += c * d.y * I.x;
      ji[1] += c * d.y * I.y;
      jr[2] += c * d.z * I.x;
      ji[2] += c * d.z * I.y;
    }
    double2 *o = J + ((int64_t)rr * nt * 7 + t) * 3;
    o[0] = make_double2(jr[0], ji[0]);
    o[1] = make_double2(jr[1], ji[1]);
    o[2] = make_double2(jr[2], ji[2]);
  }
}

constexpr int kRcsThreads = 256;
constexpr int kChunk = 256;

__global__ void __launch_bounds__(kRcsThreads)
    k_rcs(const double *pos, const double2 *J, int64_t npts, const double *theta, int ntheta,
          const double *phi, int nphi, double k, double scale, double *sigma) {
  __shared__ double sp[kChunk * 3];
  __shared__ double2 sj[kChunk * 3];
  const int rr = blockIdx.y;
  const int64_t dir = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = dir < (int64_t)ntheta * nphi;
  const int a = ok ? (int)(dir / nphi) : 0, b = ok ? (int)(dir % nphi) : 0;
  double st, ct, sph, cph;
  sincos(theta[a], &st, &ct);
  sincos(phi[b], &sph, &cph);
  const double rx = st * cph, ry = st * sph, rz = ct;
  const double tx = ct * cph, ty = ct * sph, tz = -st;
  const double2 *Jr = J + (int64_t)rr * npts * 3;
  double nr = 0, ni = 0;
  for (int64_t c0 = 0; c0 < npts; c0 += kChunk) {
    const int cnt = (int)min<int64_t>(kChunk, npts - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * 3; i += blockDim.x) {
      sp[i] = pos[c0 * 3 + i];
      sj[i] = Jr[c0 * 3 + i];
    }
    __syncthreads();
    for (int i = 0; i < cnt; ++i) {
      const double ph = k * (rx * sp[3 * i] + ry * sp[3 * i + 1] + rz * sp[3 * i + 2]);
      double s, c;
      sincos(ph, &s, &c);
      // theta_hat . J
      const double jr = tx * sj[3 * i].x + ty * sj[3 * i + 1].x + tz * sj[3 * i + 2].x;
      const double ji = tx * sj[3 * i].y + ty * sj[3 * i + 1].y + tz * sj[3 * i + 2].y;
      nr += jr * c - ji * s;
      ni += jr * s + ji * c;
    }
  }
  if (ok) sigma[(int64_t)rr * ntheta * nphi + dir] = scale * (nr * nr + ni * ni);
}

}  // namespace

void rcs_mesh(Plan *pl, MeshDev &md, int nrhs, const double2 *x, int64_t ldx, int ntheta,
              const double *theta, int nphi, const double *phi, double *sigma, hipStream_t s) {
  const HostPlan &h = md.hp;
  const int64_t nt = h.nt, npts = 7 * nt;
  // triangle -> (basis << 1 | side) per local vertex
  std::vector<int32_t> tb(3 * nt, -1);
  for (int64_t n = 0; n < h.n; ++n) {
    for (int side = 0; side < 2; ++side) {
      const int64_t t = side == 0 ? h.tp[n] : h.tm[n];
      const int32_t fv = side == 0 ? h.vp[n] : h.vm[n];
      for (int i = 0; i < 3; ++i)
        if (h.tris[3 * t + i] == fv) tb[3 * t + i] = (int32_t)((n << 1) | side);
    }
  }
  std::vector<void *> tmp;
  auto alloc = [&](size_t bytes) {
    void *p = dev_alloc(pl, bytes);
    tmp.push_back(p);
    return p;
  };
  try {
    int32_t *dtb = (int32_t *)alloc(sizeof(int32_t) * tb.size());
    double *pos = (double *)alloc(sizeof(double) * 3 * npts);
    double2 *J = (double2 *)alloc(sizeof(double2) * 3 * npts * nrhs);
    double *dth = (double *)alloc(sizeof(double) * ntheta);
    double *dph = (double *)alloc(sizeof(double) * nphi);
    const int64_t ndir = (int64_t)ntheta * nphi;
    double *dsig = (double *)alloc(sizeof(double) * ndir * nrhs);
    HIPCHECK(hipMemcpyAsync(dtb, tb.data(), sizeof(int32_t) * tb.size(), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(dth, theta, sizeof(double) * ntheta, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(dph, phi, sizeof(double) * nphi, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_point_currents, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s,
                       md.tris, md.verts, md.area, dtb, md.len, x, ldx, nrhs, nt, pos, J);
    LAUNCHCHECK();
    const double keta = h.k * kEta0;
    const double scale = keta * keta / (4.0 * kPi);
    hipLaunchKernelGGL(k_rcs, dim3((unsigned)((ndir + kRcsThreads - 1) / kRcsThreads), nrhs),
                       dim3(kRcsThreads), 0, s, pos, J, npts, dth, ntheta, dph, nphi, h.k, scale,
                       dsig);
    LAUNCHCHECK();
    HIPCHECK(hipMemcpyAsync(sigma, dsig, sizeof(double) * ndir * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  } catch (...) {
    for (void *p : tmp) dev_free(pl, p);
    throw;
  }
  for (void *p : tmp) dev_free(pl, p);
}

}  // namespace aim
