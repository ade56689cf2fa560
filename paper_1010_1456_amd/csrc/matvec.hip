// The AIM product y = Z^near x + Z^grid x (hot path).
//
// Steps, in the paper's order (Section 4.1): projection of the basis
// currents onto the grid (anterpolation), propagation (forward FFTs, Green's
// spectrum multiply, inverse FFTs on the zero-padded grid), interpolation
// back to the testing functions, plus the sparse near-zone correction, fused
// with the interpolation so y is written once. The input vector may be of a
// wider type than the arithmetic (c128 Krylov vectors feeding the c64
// operator): the narrowing happens in registers as x is read.
#include <algorithm>

#include "aim_internal.h"

namespace aim {

namespace {

template <typename T>
__device__ __forceinline__ void atomic_add_real(T *p, T v) {
  unsafeAtomicAdd(p, v);
}

// s_q[node(n, u)] += Lambda[n][q][u] x_n for every basis n, stencil node u,
// component q, right-hand side r. One thread per (n, u).
template <typename T, typename TX>
__global__ void __launch_bounds__(256)
    k_anterp(const cx<TX> *__restrict__ x, int64_t ldx, int nrhs, const T *__restrict__ lam,
             const int32_t *__restrict__ anchor_lin, const int32_t *__restrict__ soff, int64_t n,
             int K, cx<T> *__restrict__ grid, int64_t V0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t b = t / K;
  const int u = (int)(t - b * K);
  const int64_t node = (int64_t)anchor_lin[b] + soff[u];
  T w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = lam[(b * 4 + q) * K + u];
  for (int r = 0; r < nrhs; ++r) {
    const cx<TX> xv = x[(int64_t)r * ldx + b];
    const T xr = (T)xv.x, xi = (T)xv.y;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (w[q] == (T)0) continue;
      T *g = reinterpret_cast<T *>(grid + ((int64_t)(r * 4 + q)) * V0 + node);
      atomic_add_real(g, w[q] * xr);
      atomic_add_real(g + 1, w[q] * xi);
    }
  }
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// y_m = j k eta [sum_{q<3} Lambda_mq . phi_q - k^-2 Lambda_md . phi_d]
//       + sum_n Z^near_mn x_n. One 64-lane wave per row m.
template <typename T, typename TX, typename TY>
__global__ void __launch_bounds__(256)
    k_interp_near(const cx<T> *__restrict__ phi, int64_t V0, int nrhs, const T *__restrict__ lam,
                  const int32_t *__restrict__ anchor_lin, const int32_t *__restrict__ soff, int K,
                  const int32_t *__restrict__ rowptr, const int32_t *__restrict__ cols,
                  const cx<T> *__restrict__ nearv, const cx<TX> *__restrict__ x, int64_t ldx,
                  cx<TY> *__restrict__ y, int64_t ldy, int64_t n, T keta, T inv_k2) {
  using V = cx<T>;
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (m >= n) return;
  const int64_t a = anchor_lin[m];
  const int e0 = rowptr[m], e1 = rowptr[m + 1];
  for (int r = 0; r < nrhs; ++r) {
    V far;
    far.x = 0;
    far.y = 0;
    const V *ph = phi + (int64_t)(r * 4) * V0 + a;
    for (int u = lane; u < K; u += 64) {
      const int64_t o = soff[u];
      const T l0 = lam[(m * 4 + 0) * K + u], l1 = lam[(m * 4 + 1) * K + u];
      const T l2 = lam[(m * 4 + 2) * K + u], l3 = lam[(m * 4 + 3) * K + u];
      const V p0 = ph[o], p1 = ph[V0 + o], p2 = ph[2 * V0 + o], p3 = ph[3 * V0 + o];
      far.x += l0 * p0.x + l1 * p1.x + l2 * p2.x - inv_k2 * l3 * p3.x;
      far.y += l0 * p0.y + l1 * p1.y + l2 * p2.y - inv_k2 * l3 * p3.y;
    }
    V nr;
    nr.x = 0;
    nr.y = 0;
    const cx<TX> *xr = x + (int64_t)r * ldx;
    for (int e = e0 + lane; e < e1; e += 64) {
      const V z = nearv[e];
      const cx<TX> xv = xr[cols[e]];
      const T xa = (T)xv.x, xb = (T)xv.y;
      nr.x += z.x * xa - z.y * xb;
      nr.y += z.x * xb + z.y * xa;
    }
    V acc;
    acc.x = -keta * far.y + nr.x;  // j k eta * far
    acc.y = keta * far.x + nr.y;
    acc = wave_sum(acc);
    if (lane == 0) {
      cx<TY> out;
      out.x = (decltype(out.x))acc.x;
      out.y = (decltype(out.y))acc.y;
      y[(int64_t)r * ldy + m] = out;
    }
  }
}

template <typename T>
const T *lam_of(const MeshDev &md);
template <>
const double *lam_of<double>(const MeshDev &md) {
  return md.lam64;
}
template <>
const float *lam_of<float>(const MeshDev &md) {
  return md.lam32;
}
template <typename T>
const cx<T> *near_of(const MeshDev &md);
template <>
const double2 *near_of<double>(const MeshDev &md) {
  return md.near64;
}
template <>
const float2 *near_of<float>(const MeshDev &md) {
  return md.near32;
}
template <typename T>
const cx<T> *ghat_of(const MeshDev &md);
template <>
const double2 *ghat_of<double>(const MeshDev &md) {
  return md.ghat64;
}
template <>
const float2 *ghat_of<float>(const MeshDev &md) {
  return md.ghat32;
}
template <typename T>
const cx<T> *tw_of(const MeshDev &md, int d);
template <>
const double2 *tw_of<double>(const MeshDev &md, int d) {
  return md.tw64[d];
}
template <>
const float2 *tw_of<float>(const MeshDev &md, int d) {
  return md.tw32[d];
}

}  // namespace

void *work_buffer(Plan *pl, int prec, int which, size_t bytes) {
  if (pl->work_bytes[prec][which] < bytes) {
    if (pl->work[prec][which]) dev_free(pl, pl->work[prec][which]);
    pl->work[prec][which] = nullptr;
    pl->work_bytes[prec][which] = 0;
    pl->work[prec][which] = dev_alloc(pl, bytes);
    pl->work_bytes[prec][which] = bytes;
  }
  return pl->work[prec][which];
}

template <typename T, typename TX>
void far_stages(Plan *pl, MeshDev &md, int nrhs, const cx<TX> *x, int64_t ldx, int stop,
                hipStream_t s) {
  const HostPlan &h = md.hp;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int Nx = h.grid[0], Ny = h.grid[1], Nz = h.grid[2];
  const int Px = h.pad[0], Py = h.pad[1], Pz = h.pad[2];
  (void)Px;
  const int64_t F = 4 * (int64_t)nrhs;
  const int64_t V0 = (int64_t)Nx * Ny * Nz;
  const int64_t V1 = (int64_t)Nx * Ny * Pz;
  const int64_t V2 = (int64_t)Nx * Py * Pz;
  cx<T> *g0 = (cx<T> *)work_buffer(pl, prec, 0, sizeof(cx<T>) * F * V0);
  cx<T> *g1 = (cx<T> *)work_buffer(pl, prec, 1, sizeof(cx<T>) * F * V1);
  cx<T> *g2 = (cx<T> *)work_buffer(pl, prec, 2, sizeof(cx<T>) * F * V2);
  const int K = h.K;
  HIPCHECK(hipMemsetAsync(g0, 0, sizeof(cx<T>) * F * V0, s));
  {
    const int64_t threads = h.n * K;
    hipLaunchKernelGGL((k_anterp<T, TX>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       x, ldx, nrhs, lam_of<T>(md), md.anchor_lin, md.stencil_off, h.n, K, g0, V0);
    LAUNCHCHECK();
  }
  if (stop <= 1) return;
  fft_pass_contig(g0, g1, md.plan[2], Nz, Pz, F * Nx * Ny, Nz, Pz, false, tw_of<T>(md, 2), s);
  if (stop <= 2) return;
  fft_pass_strided(g1, g2, md.plan[1], Ny, Py, F * Nx, Pz, Pz, (int64_t)Ny * Pz, Pz,
                      (int64_t)Py * Pz, false, tw_of<T>(md, 1), s);
  if (stop <= 3) return;
  fft_mid_pass(g2, md.plan[0], Nx, (int)F, Py, Pz, md.H[0], md.H[1], md.H[2], ghat_of<T>(md),
                  tw_of<T>(md, 0), s);
  if (stop <= 4) return;
  fft_pass_strided(g2, g1, md.plan[1], Py, Ny, F * Nx, Pz, Pz, (int64_t)Py * Pz, Pz,
                      (int64_t)Ny * Pz, true, tw_of<T>(md, 1), s);
  if (stop <= 5) return;
  fft_pass_contig(g1, g0, md.plan[2], Pz, Nz, F * Nx * Ny, Pz, Nz, true, tw_of<T>(md, 2), s);
}

template <typename T, typename TX, typename TY>
void matvec_mesh(Plan *pl, MeshDev &md, int nrhs, const cx<TX> *x, int64_t ldx, cx<TY> *y,
                 int64_t ldy, hipStream_t s) {
  const HostPlan &h = md.hp;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  far_stages<T, TX>(pl, md, nrhs, x, ldx, 6, s);
  const cx<T> *phi = (const cx<T> *)pl->work[prec][0];
  const int64_t V0 = (int64_t)h.grid[0] * h.grid[1] * h.grid[2];
  const int rows_per_block = 4;
  const int64_t blocks = (h.n + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL((k_interp_near<T, TX, TY>), dim3((unsigned)blocks), dim3(64 * rows_per_block),
                     0, s, phi, V0, nrhs, lam_of<T>(md), md.anchor_lin, md.stencil_off, h.K,
                     md.rowptr, md.cols, near_of<T>(md), x, ldx, y, ldy, h.n,
                     (T)(h.k * kEta0), (T)(1.0 / (h.k * h.k)));
  LAUNCHCHECK();
}

template void far_stages<double, double>(Plan *, MeshDev &, int, const double2 *, int64_t, int,
                                         hipStream_t);
template void far_stages<float, float>(Plan *, MeshDev &, int, const float2 *, int64_t, int,
                                       hipStream_t);
template void far_stages<float, double>(Plan *, MeshDev &, int, const double2 *, int64_t, int,
                                        hipStream_t);
template void matvec_mesh<double, double, double>(Plan *, MeshDev &, int, const double2 *, int64_t,
                                                  double2 *, int64_t, hipStream_t);
template void matvec_mesh<float, float, float>(Plan *, MeshDev &, int, const float2 *, int64_t,
                                               float2 *, int64_t, hipStream_t);
template void matvec_mesh<float, double, double>(Plan *, MeshDev &, int, const double2 *, int64_t,
                                                 double2 *, int64_t, hipStream_t);

}  // namespace aim
