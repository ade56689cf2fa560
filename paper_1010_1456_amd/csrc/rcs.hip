// Bistatic radar cross section sigma_theta_theta (FP64).
//
// The paper measures accuracy through the VV bistatic RCS over the sphere of
// directions (Section 2.2, eq. 1). With J = sum_n I_n f_n, the radiation
// vector is N(r_hat) = int J exp(+j k r_hat . r') dS' and, for a unit incident
// field, sigma_tt = (k eta)^2 / (4 pi) |theta_hat . N|^2. Work-groups cover a
// tile of directions and a chunk of the triangles' quadrature points; each
// thread sums its points for the tile's directions, the work-group reduces,
// and the chunks' partial sums are added in a fixed order.
//
// Two ways to feed the points: aim_rcs first collapses the current onto the
// 7 quadrature points of every triangle (positions and A w J in temporary
// buffers); the allocation-free variant forms each point's position and
// current inside the kernel from the mesh and the triangle -> basis table,
// and keeps its partial sums in a fixed device array (below).
#include <cmath>
#include <mutex>

#include "aim_internal.h"
#include "geom_device.h"

namespace aim {
using namespace geo;

namespace {

// Partial sums of the allocation-free RCS: one array per GPU for the whole
// process, kRcsScratchElems double2 (16 MiB). Host code never passes this
// name to a kernel (on the host it is only a stand-in): it uses the device
// address looked up by rcs_scratch_init.
static __device__ __align__(256) double2 scratch[kRcsScratchElems];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// position and A w J of quadrature point p (tri = p / 7) of one right-hand side
__device__ __forceinline__ void point_current(const int32_t *tris, const double *verts,
                                              const double *area, const int32_t *tri_basis,
                                              const double *len, const double2 *xr, int64_t t,
                                              D3 *r, double2 *J) {
  const int64_t tri = t / 7;
  const int p = (int)(t - tri * 7);
  D3 T[3];
  for (int c = 0; c < 3; ++c) T[c] = vtx(verts, tris[3 * tri + c]);
  double w;
  *r = quad_point(T, p, &w);
  const double A = area[tri];
  double jr[3] = {0, 0, 0}, ji[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const int code = tri_basis[3 * tri + i];
    if (code < 0) continue;
    const int64_t n = code >> 1;
    const double s = (code & 1) ? -1.0 : 1.0;
    // f_n = s l / (2A) (r - v_i) on this triangle, v_i the free vertex
    const double c = s * len[n] / (2.0 * A) * A * w;
    const D3 d = *r - T[i];
    const double2 I = xr[n];
    jr[0] += c * d.x * I.x;
    ji[0] += c * d.x * I.y;
    jr[1] += c * d.y * I.x;
    ji[1] += c * d.y * I.y;
    jr[2] += c * d.z * I.x;
    ji[2] += c * d.z * I.y;
  }
  J[0] = make_double2(jr[0], ji[0]);
  J[1] = make_double2(jr[1], ji[1]);
  J[2] = make_double2(jr[2], ji[2]);
}

// per triangle quadrature point: position (3) and A w J (3 complex)
__global__ void k_point_currents(const int32_t *tris, const double *verts, const double *area,
                                 const int32_t *tri_basis, const double *len, const double2 *x,
                                 int64_t ldx, int nrhs, int64_t nt, double *pos, double2 *J) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt * 7) return;
  for (int rr = 0; rr < nrhs; ++rr) {
    D3 r;
    double2 Jp[3];
    point_current(tris, verts, area, tri_basis, len, x + (int64_t)rr * ldx, t, &r, Jp);
    if (rr == 0) {
      pos[3 * t] = r.x;
      pos[3 * t + 1] = r.y;
      pos[3 * t + 2] = r.z;
    }
    double2 *o = J + ((int64_t)rr * nt * 7 + t) * 3;
    o[0] = Jp[0];
    o[1] = Jp[1];
    o[2] = Jp[2];
  }
}

constexpr int kRcsThreads = 256;
constexpr int kDirTile = 8;      // directions per work-group
constexpr int kPtsChunk = 4096;  // quadrature points per work-group (aim_rcs)

// The points a part kernel sums: precomputed (aim_rcs) or formed in place.
struct PointsStored {
  const double *pos;
  const double2 *J;  // [nrhs][npts][3]
  __device__ void get(int rr, int64_t npts, int64_t p, D3 *r, double2 *Jp) const {
    *r = d3(pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]);
    const double2 *Jr = J + (int64_t)rr * npts * 3;
    Jp[0] = Jr[3 * p];
    Jp[1] = Jr[3 * p + 1];
    Jp[2] = Jr[3 * p + 2];
  }
};
struct PointsInPlace {
  const int32_t *tris;
  const double *verts;
  const double *area;
  const int32_t *tri_basis;
  const double *len;
  const double2 *x;
  int64_t ldx;
  __device__ void get(int rr, int64_t, int64_t p, D3 *r, double2 *Jp) const {
    point_current(tris, verts, area, tri_basis, len, x + (int64_t)rr * ldx, p, r, Jp);
  }
};

// part[(rr ndir + d) nchunk + chunk] = sum over the chunk's points of
// (theta_hat(d) . J) exp(+j k r_hat(d) . r); chunk = blockIdx.y covers
// points [chunk * per_chunk, (chunk + 1) * per_chunk)
template <class PTS>
__global__ void __launch_bounds__(kRcsThreads)
    k_rcs_part(PTS pts, int64_t npts, int64_t per_chunk, const double *theta, int ntheta,
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
  const int64_t p0 = (int64_t)blockIdx.y * per_chunk;
  const int64_t p1 = min(p0 + per_chunk, npts);
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kRcsThreads) {
    D3 r;
    double2 Jp[3];
    pts.get(rr, npts, p, &r, Jp);
    const double2 jx = Jp[0], jy = Jp[1], jz = Jp[2];
#pragma unroll
    for (int q = 0; q < kDirTile; ++q) {
      const double *o = dir[q];
      double s, c;
      sincos(k * (o[0] * r.x + o[1] * r.y + o[2] * r.z), &s, &c);
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

void rcs_prepare_mesh(Plan *pl, MeshDev &md, hipStream_t s) {
  const HostPlan &h = md.hp;
  std::vector<int32_t> tb(3 * h.nt, -1);
  for (int64_t n = 0; n < h.n; ++n) {
    for (int side = 0; side < 2; ++side) {
      const int64_t t = side == 0 ? h.tp[n] : h.tm[n];
      const int32_t fv = side == 0 ? h.vp[n] : h.vm[n];
      for (int i = 0; i < 3; ++i)
        if (h.tris[3 * t + i] == fv) tb[3 * t + i] = (int32_t)((n << 1) | side);
    }
  }
  md.tri_basis = (int32_t *)dev_alloc(pl, sizeof(int32_t) * tb.size());
  HIPCHECK(hipMemcpyAsync(md.tri_basis, tb.data(), sizeof(int32_t) * tb.size(),
                          hipMemcpyHostToDevice, s));
  HIPCHECK(hipStreamSynchronize(s));  // tb is a host temporary
}

void rcs_scratch_init() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(AIM_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void *p = nullptr;
  HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(AIM_ERR_HIP, "no device address for the RCS scratch array");
  g_scratch_ptr[dev] = p;
}

void *rcs_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

void rcs_mesh(Plan *pl, MeshDev &md, int nrhs, const double2 *x, int64_t ldx, int ntheta,
              const double *theta, int nphi, const double *phi, double *sigma, hipStream_t s) {
  const HostPlan &h = md.hp;
  const int64_t nt = h.nt, npts = 7 * nt;
  std::vector<void *> tmp;
  auto alloc = [&](size_t bytes) {
    void *p = dev_alloc(pl, bytes);
    tmp.push_back(p);
    return p;
  };
  try {
    double *pos = (double *)alloc(sizeof(double) * 3 * npts);
    double2 *J = (double2 *)alloc(sizeof(double2) * 3 * npts * nrhs);
    double *dth = (double *)alloc(sizeof(double) * ntheta);
    double *dph = (double *)alloc(sizeof(double) * nphi);
    const int64_t ndir = (int64_t)ntheta * nphi;
    double *dsig = (double *)alloc(sizeof(double) * ndir * nrhs);
    HIPCHECK(hipMemcpyAsync(dth, theta, sizeof(double) * ntheta, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(dph, phi, sizeof(double) * nphi, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_point_currents, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s,
                       md.tris, md.verts, md.area, md.tri_basis, md.len, x, ldx, nrhs, nt, pos, J);
    LAUNCHCHECK();
    const double keta = h.k * kEta0;
    const double scale = keta * keta / (4.0 * kPi);
    const int nchunk = (int)((npts + kPtsChunk - 1) / kPtsChunk);
    double2 *part = (double2 *)alloc(sizeof(double2) * (size_t)ndir * nrhs * nchunk);
    hipLaunchKernelGGL((k_rcs_part<PointsStored>),
                       dim3((unsigned)((ndir + kDirTile - 1) / kDirTile), (unsigned)nchunk, nrhs),
                       dim3(kRcsThreads), 0, s, PointsStored{pos, J}, npts, (int64_t)kPtsChunk,
                       dth, ntheta, dph, nphi, h.k, nchunk, part);
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

void rcs_mesh_noalloc(MeshDev &md, int nrhs, const double2 *x, int64_t ldx, int ntheta,
                      const double *theta, int nphi, const double *phi, double *sigma,
                      double2 *part, hipStream_t s) {
  const HostPlan &h = md.hp;
  const int64_t npts = 7 * h.nt;
  const int64_t ndir = (int64_t)ntheta * nphi;
  const int64_t slots = ndir * nrhs;  // partial sums needed per chunk
  if (slots > kRcsScratchElems)
    throw Error(AIM_ERR_ARG, "aim_rcs_noalloc: ntheta * nphi * nrhs = " + std::to_string(slots) +
                                 " exceeds its fixed scratch of " +
                                 std::to_string(kRcsScratchElems) + " partial sums");
  // as many point chunks as aim_rcs uses, fewer if the scratch cannot hold them
  int64_t nchunk = (npts + kPtsChunk - 1) / kPtsChunk;
  if (nchunk * slots > kRcsScratchElems) nchunk = kRcsScratchElems / slots;
  if (nchunk < 1) nchunk = 1;
  const int64_t per_chunk = (npts + nchunk - 1) / nchunk;
  const double keta = h.k * kEta0;
  const double scale = keta * keta / (4.0 * kPi);
  hipLaunchKernelGGL((k_rcs_part<PointsInPlace>),
                     dim3((unsigned)((ndir + kDirTile - 1) / kDirTile), (unsigned)nchunk, nrhs),
                     dim3(kRcsThreads), 0, s,
                     PointsInPlace{md.tris, md.verts, md.area, md.tri_basis, md.len, x, ldx}, npts,
                     per_chunk, theta, ntheta, phi, nphi, h.k, (int)nchunk, part);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_rcs_reduce, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, s, part,
                     (int)nchunk, slots, scale, sigma);
  LAUNCHCHECK();
}

}  // namespace aim
