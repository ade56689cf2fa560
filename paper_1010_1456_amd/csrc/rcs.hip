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
constexpr int kDirTile = 8;      // directions per work-group
constexpr int kPtsChunk = 4096;  // quadrature points per work-group

// part[(rr ndir + d) nchunk + chunk] = sum over the chunk's points of
// (theta_hat(d) . J) exp(+j k r_hat(d) . r)
__global__ void __launch_bounds__(kRcsThreads)
    k_rcs_part(const double *pos, const double2 *J, int64_t npts, const double *theta, int ntheta,
               const double *phi, int nphi, double k, int nchunk, double2 *part) {
  __shared__ double dir[kDirTile][6];  // r_hat, theta_hat
  __shared__ double red[kRcsThreads / 64][2 * kDirTile];
  const int rr = blockIdx.z;
  const int64_t ndir = (int64_t)ntheta * nphi;
  const int64_t d0 = (int64_t)blockIdx.x * kDirTile;
  if (threadIdx.x < kDirTile) {
    const int64_t d = d0 + threadIdx.x;
    double st = 0, ct = 1, sph = 0, cph = 1;
    if (d < ndir) {
      sincos(theta[d / nphi], &st, &ct);
      sincos(phi[d % nphi], &sph, &cph);
    }
    double *o = dir[threadIdx.x];
    o[0] = st * cph;
    o[1] = st * sph;
    o[2] = ct;
    o[3] = ct * cph;
    o[4] = ct * sph;
    o[5] = -st;
  }
  __syncthreads();
  double nr[kDirTile], ni[kDirTile];
#pragma unroll
  for (int q = 0; q < kDirTile; ++q) nr[q] = ni[q] = 0;
  const double2 *Jr = J + (int64_t)rr * npts * 3;
  const int64_t p0 = (int64_t)blockIdx.y * kPtsChunk;
  const int64_t p1 = min(p0 + kPtsChunk, npts);
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kRcsThreads) {
    const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
    const double2 jx = Jr[3 * p], jy = Jr[3 * p + 1], jz = Jr[3 * p + 2];
#pragma unroll
    for (int q = 0; q < kDirTile; ++q) {
      const double *o = dir[q];
      double s, c;
      sincos(k * (o[0] * x + o[1] * y + o[2] * z), &s, &c);
      const double jr = o[3] * jx.x + o[4] * jy.x + o[5] * jz.x;  // theta_hat . J
      const double ji = o[3] * jx.y + o[4] * jy.y + o[5] * jz.y;
      nr[q] += jr * c - ji * s;
      ni[q] += jr * s + ji * c;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kDirTile; ++q) {
    for (int off = 32; off > 0; off >>= 1) {
      nr[q] += __shfl_xor(nr[q], off, 64);
      ni[q] += __shfl_xor(ni[q], off, 64);
    }
    if (lane == 0) {
      red[w][2 * q] = nr[q];
      red[w][2 * q + 1] = ni[q];
    }
  }
  __syncthreads();
  if (threadIdx.x < kDirTile && d0 + threadIdx.x < ndir) {
    double a = 0, b = 0;
    for (int i = 0; i < kRcsThreads / 64; ++i) {
      a += red[i][2 * threadIdx.x];
      b += red[i][2 * threadIdx.x + 1];
    }
    part[((int64_t)rr * ndir + d0 + threadIdx.x) * nchunk + blockIdx.y] = make_double2(a, b);
  }
}

// sigma[rr ndir + d] = scale |sum over chunks of part|^2 (chunks in order)
__global__ void k_rcs_reduce(const double2 *part, int nchunk, int64_t count, double scale,
                             double *sigma) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  double a = 0, b = 0;
  for (int c = 0; c < nchunk; ++c) {
    const double2 v = part[t * nchunk + c];
    a += v.x;
    b += v.y;
  }
  sigma[t] = scale * (a * a + b * b);
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
    const int nchunk = (int)((npts + kPtsChunk - 1) / kPtsChunk);
    double2 *part = (double2 *)alloc(sizeof(double2) * (size_t)ndir * nrhs * nchunk);
    hipLaunchKernelGGL(k_rcs_part,
                       dim3((unsigned)((ndir + kDirTile - 1) / kDirTile), (unsigned)nchunk, nrhs),
                       dim3(kRcsThreads), 0, s, pos, J, npts, dth, ntheta, dph, nphi, h.k, nchunk,
                       part);
    LAUNCHCHECK();
    hipLaunchKernelGGL(k_rcs_reduce, dim3((unsigned)((ndir * nrhs + 255) / 256)), dim3(256), 0, s,
                       part, nchunk, ndir * nrhs, scale, dsig);
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
