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
#include "fft_map.h"

namespace aim {

namespace {

// Gather form of anterpolation: grid node v sums Lambda_T[e] x_{col[e]} over
// its entries, so every node (also empty ones) is written exactly once, with
// no atomics and no clearing pass, in a fixed order (bitwise reproducible).
// Each 64-lane wave owns npw <= 64 consecutive nodes (fewer where nodes hold
// many entries, so that a wave's entries stay few), whose entries are contiguous:
// the wave loads them epl * 64 at a time (coalesced; every lane has epl
// independent gathers in flight), each lane forming its entries' four products
// in LDS; then the 64 / npw lanes of each node sum every (64 / npw)-th of its
// slots and combine their sums by exchanges within the group (one right-hand
// side per blockIdx.y). Entries per lane
// per chunk: 2 (measured on the sphere over the occupied nodes: 1 or 4 is
// slower for float, 1 for double by 30%)
template <typename T>
constexpr int anterp_epl() {
  return 2;
}
// occupied nodes per wave of the 3-D projection
// occupied nodes per wave of the gather: candidates timed at set-up (on the
// sphere: 64 0.079 ms, 32 0.067, 16 0.058, 8 0.056 for c64; 16 best for c128)
constexpr int kGatherNpwCand[3] = {8, 16, 32};
// With occ (the occupied nodes, increasing) the wave walks npw consecutive
// occupied nodes instead: node_ptr is then their compacted entry ranges, V0
// their count, and node i is written at grid index occ[i] of fields of Vg
// nodes; the other nodes are left untouched (zero in the caller's buffer).
template <typename T, typename TX>
__global__ void __launch_bounds__(256)
    k_anterp_gather(const cx<TX> *__restrict__ x, int64_t ldx, int nrhs,
                    const int32_t *__restrict__ node_ptr, const int32_t *__restrict__ occ,
                    const int32_t *__restrict__ ent_col, const T *__restrict__ lamT,
                    cx<T> *__restrict__ grid, int64_t V0, int64_t Vg, int npw) {
  constexpr int kEpl = anterp_epl<T>();
  constexpr int C = 64 * kEpl;      // entries per chunk
  __shared__ cx<T> slot[4][C][4];  // [wave][entry][q]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t v0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + w) * npw;
  if (v0 >= V0) return;  // whole wave exits; no block-wide barrier is used
  // G = 64 / npw lanes per node (npw divides 64, checked by the launcher):
  // lane = node * G + sub
  const int G = 64 / npw, sub = lane & (G - 1);
  const int64_t v = v0 + lane / G;
  const bool ok = v < V0;
  const int64_t vend = (v0 + npw < V0) ? v0 + npw : V0;
  const int e0 = ok ? node_ptr[v] : 0, e1 = ok ? node_ptr[v + 1] : 0;
  const int w0 = node_ptr[v0], w1 = node_ptr[vend];
  {
    const int r = blockIdx.y;  // right-hand side
    const cx<TX> *xr = x + (int64_t)r * ldx;
    T a[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int c0 = w0; c0 < w1; c0 += C) {
      int col[kEpl];
#pragma unroll
      for (int u = 0; u < kEpl; ++u) {
        const int e = c0 + u * 64 + lane;
        col[u] = e < w1 ? ent_col[e] : -1;
      }
#pragma unroll
      for (int u = 0; u < kEpl; ++u) {
        const int e = c0 + u * 64 + lane;
        if (col[u] >= 0) {
          const cx<TX> xv = xr[col[u]];
          const T xa = (T)xv.x, xb = (T)xv.y;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T wq = lamT[(int64_t)e * 4 + q];
            cx<T> p;
            p.x = wq * xa;
            p.y = wq * xb;
            slot[w][u * 64 + lane][q] = p;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int lo = (e0 > c0 ? e0 : c0) - c0, hi = (e1 < c0 + C ? e1 : c0 + C) - c0;
      for (int k = lo + sub; k < hi; k += G) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const cx<T> p = slot[w][k][q];
          a[q][0] += p.x;
          a[q][1] += p.y;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int off = 1; off < G; off <<= 1)  // the group's partial sums, fixed order
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q][0] += __shfl_xor(a[q][0], off, 64);
        a[q][1] += __shfl_xor(a[q][1], off, 64);
      }
    if (ok && sub == 0) {
      const int64_t node = occ ? (int64_t)occ[v] : v;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cx<T> o;
        o.x = a[q][0];
        o.y = a[q][1];
        grid[((int64_t)(r * 4 + q)) * Vg + node] = o;
      }
    }
  }
}

template <typename T>
__global__ void k_zero(cx<T> *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i].x = p[i].y = 0;
}

// thin [F][Pz][A] grid -> plain [F][A][Pz] (inspection)
template <typename T>
__global__ void k_kz_inner(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int64_t F,
                           int64_t A, int Pz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= F * A * Pz) return;
  const int kz = (int)(t % Pz);
  const int64_t a = (t / Pz) % A, f = t / (Pz * A);
  out[t] = in[(f * Pz + kz) * A + a];
}

// kz-blocked [F][Pz/blk][Nx][Py][blk] grid -> plain [F][Nx][Py][Pz] (inspection)
template <typename T>
__global__ void k_unblock(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int64_t F, int Nx,
                          int Py, int Pz, int blk, int64_t fstride) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = F * Nx * Py * Pz;
  if (t >= tot) return;
  const int kz = (int)(t % Pz);
  const int ky = (int)((t / Pz) % Py);
  const int x = (int)((t / ((int64_t)Py * Pz)) % Nx);
  const int64_t f = t / ((int64_t)Nx * Py * Pz);
  out[t] = in[f * fstride + ((int64_t)(kz / blk) * Nx + x) * Py * blk + (int64_t)ky * blk + kz % blk];
}

template <typename V>
__device__ __forceinline__ V half_wave_sum(V v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 32);
    v.y += __shfl_xor(v.y, off, 32);
  }
  return v;
}

// y_m = j k eta [sum_{q<3} Lambda_mq . phi_q - k^-2 Lambda_md . phi_d]
//       + sum_n Z^near_mn x_n. One 32-lane half-wave per row m.
constexpr int kNearUnroll = 4;

// RB right-hand sides per grid row (blockIdx.y): the stencil weights, the
// near-zone entries and their columns are loaded once for the RB products.
// CF (combined field): y^far = keta j [sum_q Lambda_q^T phi_q - inv_k2
// Lambda_d^T phi_d] - eta_h sum_e W_e^T phi_e, with keta = alpha k eta and
// eta_h = (1 - alpha) eta; the curl weights W test the vector potential's curl.
template <typename T, typename TX, typename TY, int RB, bool CF>
__global__ void __launch_bounds__(256)
    k_interp_near(const cx<T> *__restrict__ phi, int64_t nf, int nrhs, const T *__restrict__ lam,
                  const T *__restrict__ curl, const int32_t *__restrict__ anchor_lin,
                  const int32_t *__restrict__ soff, int K, const int32_t *__restrict__ rowptr,
                  const int32_t *__restrict__ cols, const cx<T> *__restrict__ nearv,
                  const cx<TX> *__restrict__ x, int64_t ldx, cx<TY> *__restrict__ y, int64_t ldy,
                  int64_t n, T keta, T inv_k2, T eta_h) {
  using V = cx<T>;
  const int lane = threadIdx.x & 31;
  const int64_t m = (int64_t)blockIdx.x * (blockDim.x >> 5) + (threadIdx.x >> 5);
  if (m >= n) return;  // both rows of a wave exit together or each half runs alone
  const int64_t a = anchor_lin[m];
  const int e0 = rowptr[m], e1 = rowptr[m + 1];
  const int r0 = blockIdx.y * RB;  // first right-hand side of this row
  V far[RB], nr[RB], fk[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
    far[rb].x = far[rb].y = nr[rb].x = nr[rb].y = fk[rb].x = fk[rb].y = 0;
  for (int u = lane; u < K; u += 32) {
    const int64_t o = a + soff[u];
    const T l0 = lam[(m * 4 + 0) * K + u], l1 = lam[(m * 4 + 1) * K + u];
    const T l2 = lam[(m * 4 + 2) * K + u], l3 = lam[(m * 4 + 3) * K + u];
    T w0 = 0, w1 = 0, w2 = 0;
    if (CF) {
      w0 = curl[(m * 3 + 0) * K + u];
      w1 = curl[(m * 3 + 1) * K + u];
      w2 = curl[(m * 3 + 2) * K + u];
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const V *ph = phi + o * nf + (r0 + rb) * 4;  // fields interleaved per node
      const V p0 = ph[0], p1 = ph[1], p2 = ph[2], p3 = ph[3];
      far[rb].x += l0 * p0.x + l1 * p1.x + l2 * p2.x - inv_k2 * l3 * p3.x;
      far[rb].y += l0 * p0.y + l1 * p1.y + l2 * p2.y - inv_k2 * l3 * p3.y;
      if (CF) {
        fk[rb].x += w0 * p0.x + w1 * p1.x + w2 * p2.x;
        fk[rb].y += w0 * p0.y + w1 * p1.y + w2 * p2.y;
      }
    }
  }
  // kNearUnroll entries per lane per pass, all gathers issued before any is
  // used (rows hold ~80 entries: one pass of dependent loads, not three)
  for (int eb = e0 + lane; eb < e1; eb += 32 * kNearUnroll) {
    V z[kNearUnroll];
    int c[kNearUnroll];
#pragma unroll
    for (int k = 0; k < kNearUnroll; ++k) {
      const int e = eb + 32 * k;
      const bool in = e < e1;
      c[k] = in ? cols[e] : 0;
      if (in) {
        z[k] = nearv[e];
      } else {
        z[k].x = 0;
        z[k].y = 0;
      }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const cx<TX> *xr = x + (int64_t)(r0 + rb) * ldx;
#pragma unroll
      for (int k = 0; k < kNearUnroll; ++k) {
        const cx<TX> xv = xr[c[k]];
        const T xa = (T)xv.x, xb = (T)xv.y;
        nr[rb].x += z[k].x * xa - z[k].y * xb;
        nr[rb].y += z[k].x * xb + z[k].y * xa;
      }
    }
  }
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    V acc;
    acc.x = -keta * far[rb].y + nr[rb].x;  // j k eta * far
    acc.y = keta * far[rb].x + nr[rb].y;
    if (CF) {
      acc.x -= eta_h * fk[rb].x;
      acc.y -= eta_h * fk[rb].y;
    }
    acc = half_wave_sum(acc);
    if (lane == 0) {
      cx<TY> out;
      out.x = (decltype(out.x))acc.x;
      out.y = (decltype(out.y))acc.y;
      y[(int64_t)(r0 + rb) * ldy + m] = out;
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
const T *curl_of(const MeshDev &md);
template <>
const double *curl_of<double>(const MeshDev &md) {
  return md.curl64;
}
template <>
const float *curl_of<float>(const MeshDev &md) {
  return md.curl32;
}
template <typename T>
const T *plane_lam_of(const MeshDev &md);
template <>
const double *plane_lam_of<double>(const MeshDev &md) {
  return md.plane_lam64;
}
template <>
const float *plane_lam_of<float>(const MeshDev &md) {
  return md.plane_lam32;
}
template <typename T>
const T *lamT_of(const MeshDev &md);
template <>
const double *lamT_of<double>(const MeshDev &md) {
  return md.lamT64;
}
template <>
const float *lamT_of<float>(const MeshDev &md) {
  return md.lamT32;
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
const cx<T> *ghat2d_of(const MeshDev &md);
template <>
const double2 *ghat2d_of<double>(const MeshDev &md) {
  return md.ghat2d64;
}
template <>
const float2 *ghat2d_of<float>(const MeshDev &md) {
  return md.ghat2d32;
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

// a per-mesh grid buffer of `bytes` (grown on demand) that is zero wherever
// the kernels writing it never write
template <typename T>
static cx<T> *zeroed_buffer(Plan *pl, void *(&buf)[2], size_t (&have)[2], size_t bytes,
                            hipStream_t s) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  if (have[prec] < bytes) {
    if (buf[prec]) dev_free(pl, buf[prec]);
    buf[prec] = nullptr;
    have[prec] = 0;
    buf[prec] = dev_alloc(pl, bytes);
    have[prec] = bytes;
    ++pl->work_gen;
    const int64_t n = (int64_t)(bytes / sizeof(cx<T>));
    hipLaunchKernelGGL((k_zero<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (cx<T> *)buf[prec], n);
    LAUNCHCHECK();
  }
  return (cx<T> *)buf[prec];
}
// the mesh's projected source grid in `layout` (1: 3-D grid [F][V0], 2: the
// scatterer's plane [F][Nx Ny]), zero where no projection entry lands. The
// projection writes the occupied nodes only, so a buffer last written in the
// other layout (the full 3-D inspection of a planar scatterer, or the plane
// after it) is cleared first.
template <typename T>
static cx<T> *src_buffer(Plan *pl, MeshDev &md, size_t bytes, int layout, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const size_t had = md.src_bytes[prec];
  cx<T> *p = zeroed_buffer<T>(pl, md.src, md.src_bytes, bytes, s);
  if (md.src_bytes[prec] == had && md.src_layout[prec] != layout) {  // not just zeroed
    const int64_t n = (int64_t)(had / sizeof(cx<T>));
    hipLaunchKernelGGL((k_zero<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    LAUNCHCHECK();
  }
  md.src_layout[prec] = layout;
  return p;
}

void *work_buffer(Plan *pl, int lane, int prec, int which, size_t bytes, hipStream_t s) {
  void *(&work)[3] = pl->work[lane][prec];
  size_t(&have)[3] = pl->work_bytes[lane][prec];
  if (have[which] < bytes) {
    if (work[which]) dev_free(pl, work[which]);
    work[which] = nullptr;
    have[which] = 0;
    work[which] = dev_alloc(pl, bytes);
    have[which] = bytes;
    ++pl->work_gen;
    if (which == 0) {
      // the propagated fields: the inverse z pass writes the occupied lines
      // only and the interpolation multiplies the others by zero weights, so
      // they must hold finite values
      if (prec == 0) {
        const int64_t n = (int64_t)(bytes / sizeof(double2));
        hipLaunchKernelGGL((k_zero<double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (double2 *)work[which], n);
      } else {
        const int64_t n = (int64_t)(bytes / sizeof(float2));
        hipLaunchKernelGGL((k_zero<float>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (float2 *)work[which], n);
      }
      LAUNCHCHECK();
    }
  }
  return work[which];
}

template <typename T, typename TX>
void far_stages(Plan *pl, MeshDev &md, int nrhs, const cx<TX> *x, int64_t ldx, int stop,
                hipStream_t s, hipEvent_t *ev, bool full3d, StageView *views) {
  auto mark = [&](int i) {
    if (ev) HIPCHECK(hipEventRecord(ev[i], s));
  };
  // records where stage st left its output: plain view [F][A][Z] with strides
  auto view = [&](int st, const void *p, int64_t A, int64_t Z, int64_t fs, int64_t as,
                  int64_t zs) {
    if (!views) return;
    StageView &v = views[st];
    v = StageView{};
    v.p = p;
    v.kind = 1;
    v.F = 4 * (int64_t)nrhs;
    v.A = A;
    v.Z = Z;
    v.fs = fs;
    v.as = as;
    v.zs = zs;
  };
  if (views)
    for (int i = 0; i < AIM_NSTAGE; ++i) views[i] = StageView{};
  const HostPlan &h = md.hp;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int Nx = h.grid[0], Ny = h.grid[1], Nz = h.grid[2];
  const int Px = h.pad[0], Py = h.pad[1], Pz = h.pad[2];
  (void)Px;
  const int64_t F = 4 * (int64_t)nrhs;
  const int64_t V0 = (int64_t)Nx * Ny * Nz;
  const int blk = kGridBlock<T>;
  const int npw = md.gather_npw[prec];
  if (npw < 1 || npw > 64 || 64 % npw != 0)
    throw Error(AIM_ERR_ARG, "projection gather: nodes per wave must divide 64");
  if (md.planar_z >= 0 && !full3d) {
    // every source on the plane z = planar_z, and only that plane weighted by
    // the interpolation: the plane alone, g0 = [F][Nx][Ny], 2-D propagation
    // (y passes, x pass with the 2-D spectrum)
    const int64_t A1 = (int64_t)Nx * Ny, V2 = (int64_t)Nx * Py;
    cx<T> *g0 = (cx<T> *)work_buffer(pl, md.lane, prec, 0, sizeof(cx<T>) * F * A1, s);
    cx<T> *g2 = (cx<T> *)work_buffer(pl, md.lane, prec, 2, sizeof(cx<T>) * F * V2, s);
    cx<T> *gs = src_buffer<T>(pl, md, sizeof(cx<T>) * F * A1, 2, s);
    mark(0);
    const int64_t no = md.n_plane_occ;
    if (no > 0) {
      hipLaunchKernelGGL((k_anterp_gather<T, TX>),
                         dim3((unsigned)((no + 4 * npw - 1) / (4 * npw)), nrhs),
                         dim3(256), 0, s, x, ldx, nrhs, md.plane_occ_ptr, md.plane_occ,
                         md.ent_col, lamT_of<T>(md), gs, no, A1, npw);
      LAUNCHCHECK();
    }
    mark(1);
    view(1, gs, Nx, Ny, A1, Ny, 1);
    if (stop <= 1) return;
    mark(2);
    fft_pass_contig(gs, g2, md.plan[1], Ny, Py, F * Nx, fftk::contig_map(Ny), fftk::contig_map(Py),
                    false, tw_of<T>(md, 1), s);
    mark(3);
    view(3, g2, Nx, Py, V2, Py, 1);
    if (stop <= 3) return;
    fft_mid_pass(g2, md.plan[0], Nx, (int)F, Py, 1, md.H[0], md.H[1], 1, ghat2d_of<T>(md),
                 tw_of<T>(md, 0), 0, V2, md.x_row[prec], s);
    mark(4);
    view(4, g2, Nx, Py, V2, Py, 1);
    if (stop <= 4) return;
    // into the field-interleaved plane [Nx][Ny][F] the interpolation reads
    fft_pass_contig(g2, g0, md.plan[1], Py, Ny, F * Nx, fftk::fields_inner(F, (int64_t)Nx * Py, Py, 1),
                    fftk::fields_inner(F, 1, (int64_t)Ny * F, F), true, tw_of<T>(md, 1), s);
    mark(5);
    mark(6);
    view(6, g0, Nx, Ny, 1, (int64_t)Ny * F, F);
    return;
  }
  if (thin_layout<T>(Pz)) {
    // few kz (a flat scatterer): kz-outer layouts g1 [F][Pz][Nx][Ny] and
    // g2 [F][Pz][Nx][Py], no row padding; the y lines are contiguous, the x
    // pass tiles consecutive ky
    const int64_t A1 = (int64_t)Nx * Ny, V1 = Pz * A1, V2 = (int64_t)Pz * Nx * Py;
    cx<T> *g0 = (cx<T> *)work_buffer(pl, md.lane, prec, 0, sizeof(cx<T>) * F * V0, s);
    cx<T> *g1 = (cx<T> *)work_buffer(pl, md.lane, prec, 1, sizeof(cx<T>) * F * V1, s);
    cx<T> *g2 = (cx<T> *)work_buffer(pl, md.lane, prec, 2, sizeof(cx<T>) * F * V2, s);
    cx<T> *gs = src_buffer<T>(pl, md, sizeof(cx<T>) * F * V0, 1, s);
    mark(0);
    if (md.n_occ > 0) {
      hipLaunchKernelGGL((k_anterp_gather<T, TX>),
                         dim3((unsigned)((md.n_occ + 4 * npw - 1) / (4 * npw)), nrhs),
                         dim3(256), 0, s, x, ldx, nrhs, md.occ_ptr, md.occ, md.ent_col,
                         lamT_of<T>(md), gs, md.n_occ, V0, npw);
      LAUNCHCHECK();
    }
    mark(1);
    view(1, gs, A1, Nz, V0, Nz, 1);
    if (stop <= 1) return;
    fft_pass_contig(gs, g1, md.plan[2], Nz, Pz, F * A1, fftk::contig_map(Nz),
                    fftk::contig_map(A1, V1, 1, A1), false, tw_of<T>(md, 2), s);
    mark(2);
    view(2, g1, A1, Pz, V1, 1, A1);
    if (stop <= 2) return;
    fft_pass_contig(g1, g2, md.plan[1], Ny, Py, F * Pz * Nx, fftk::contig_map(Ny),
                    fftk::contig_map(Py), false, tw_of<T>(md, 1), s);
    mark(3);
    view(3, g2, (int64_t)Nx * Py, Pz, V2, 1, (int64_t)Nx * Py);
    if (stop <= 3) return;
    fft_mid_pass(g2, md.plan[0], Nx, (int)F, Py, Pz, md.H[0], md.H[1], md.H[2], ghat_of<T>(md),
                 tw_of<T>(md, 0), 0, V2, md.x_row[prec], s);
    mark(4);
    view(4, g2, (int64_t)Nx * Py, Pz, V2, 1, (int64_t)Nx * Py);
    if (stop <= 4) return;
    fft_pass_contig(g2, g1, md.plan[1], Py, Ny, F * Pz * Nx, fftk::contig_map(Py),
                    fftk::contig_map(Ny), true, tw_of<T>(md, 1), s);
    mark(5);
    view(5, g1, A1, Pz, V1, 1, A1);
    if (stop <= 5) return;
    if (full3d) {  // inspection: every line
      fft_pass_contig(g1, g0, md.plan[2], Pz, Nz, F * A1, fftk::contig_map(A1, V1, 1, A1),
                      fftk::contig_map(Nz), true, tw_of<T>(md, 2), s);
    } else {  // the lines the interpolation reads
      // into the field-interleaved grid [Nx][Ny][Nz][F]
      const int64_t nl = md.n_occ_lines;
      fft_pass_contig(g1, g0, md.plan[2], Pz, Nz, F * nl,
                      fftk::fields_inner(F, V1, 1, A1, md.occ_lines, nl),
                      fftk::fields_inner(F, 1, (int64_t)Nz * F, F, md.occ_lines, nl), true,
                      tw_of<T>(md, 2), s);
      view(6, g0, A1, Nz, 1, (int64_t)Nz * F, F);
    }
    mark(6);
    return;
  }
  const int Pzs = (Pz + blk - 1) / blk * blk;  // z rows padded to 128-byte multiples
  const int64_t V1 = (int64_t)Nx * Ny * Pzs;
  const int64_t V2 = (int64_t)Nx * Py * ((Pz + blk - 1) / blk * blk);  // kz-blocked
  cx<T> *g0 = (cx<T> *)work_buffer(pl, md.lane, prec, 0, sizeof(cx<T>) * F * V0, s);
  cx<T> *g1 = (cx<T> *)work_buffer(pl, md.lane, prec, 1, sizeof(cx<T>) * F * V1, s);
  cx<T> *g2 = (cx<T> *)work_buffer(pl, md.lane, prec, 2, sizeof(cx<T>) * F * V2, s);
  const fftk::LineMap m1 = fftk::plain_map((int64_t)Ny * Pzs, Pzs);
  const fftk::LineMap m2 = fftk::blocked_map(V2, Nx, Py, blk);
  cx<T> *gz = g1;  // forward z output, forward y input
  mark(0);
  // projection fused with the forward z pass: the projected grid is never
  // stored (except for inspection, or for FFT lengths without a fused kernel).
  // The variant is tuned on one right-hand side and walks the right-hand
  // sides in turn, so several take the two-launch form (right-hand sides in
  // parallel).
  if (stop <= 1 || !md.fuse_proj[prec] || nrhs > 1 ||
      !anterp_fftz(x, ldx, nrhs, md.node_ptr, md.ent_col, lamT_of<T>(md), Nz, (int64_t)Nx * Ny, g1,
                   Pzs, (int64_t)Nx * Ny * Pzs, tw_of<T>(md, 2), md.plan[2], s)) {
    cx<T> *gs = src_buffer<T>(pl, md, sizeof(cx<T>) * F * V0, 1, s);
    if (md.n_occ > 0) {
      hipLaunchKernelGGL((k_anterp_gather<T, TX>),
                         dim3((unsigned)((md.n_occ + 4 * npw - 1) / (4 * npw)), nrhs),
                         dim3(256), 0, s, x, ldx, nrhs, md.occ_ptr, md.occ, md.ent_col,
                         lamT_of<T>(md), gs, md.n_occ, V0, npw);
      LAUNCHCHECK();
    }
    mark(1);
    view(1, gs, (int64_t)Nx * Ny, Nz, V0, Nz, 1);
    if (stop <= 1) return;
    if (full3d) {  // inspection: every line, into g1
      fft_pass_contig(gs, g1, md.plan[2], Nz, Pz, F * Nx * Ny, fftk::contig_map(Nz),
                      fftk::contig_map(Pzs), false, tw_of<T>(md, 2), s);
    } else {  // the occupied lines into the mesh's zeroed buffer (the others stay zero)
      const int64_t nl = md.n_occ_lines, A1 = (int64_t)Nx * Ny;
      gz = zeroed_buffer<T>(pl, md.fz, md.fz_bytes, sizeof(cx<T>) * F * V1, s);
      fft_pass_contig(gs, gz, md.plan[2], Nz, Pz, F * nl,
                      fftk::select_lines(fftk::contig_map(Nz), md.occ_lines, nl, A1, md.occ_zrange),
                      fftk::select_lines(fftk::contig_map(Pzs), md.occ_lines, nl, A1), false,
                      tw_of<T>(md, 2), s);
    }
  } else {
    mark(1);
  }
  mark(2);
  view(2, gz, (int64_t)Nx * Ny, Pz, (int64_t)Nx * Ny * Pzs, Pzs, 1);
  if (stop <= 2) return;
  // y passes: rows outside a plane's occupied y range are zero on input
  // (forward) and never read on output (inverse); inspection keeps every row
  const fftk::LineMap m1y = full3d ? m1 : fftk::with_range(m1, md.occ_yrange, Nx);
  auto blocked_view = [&](int st) {
    if (!views) return;
    StageView &v = views[st];
    v = StageView{};
    v.p = g2;
    v.kind = 2;
    v.F = F;
    v.A = (int64_t)Nx * Py;
    v.Z = Pz;
    v.Nx = Nx;
    v.Py = Py;
    v.blk = blk;
    v.fstride = V2;
  };
  // the y, x and y passes pipelined over field groups (tuned at set-up) when
  // the product runs through; the stage boundaries then fall together (the
  // forward y step carries the time of all three)
  const int G = md.xy_groups[prec];
  if (stop >= 6 && !full3d && G > 1 && F % G == 0 &&
      xy_pipeline_available(md.plan[0], md.plan[1])) {
    fft_xy_pipeline(gz, g2, g1, md.plan[0], Nx, Ny, (int)F, G, Py, Pz, md.H[1], md.H[2],
                    ghat_of<T>(md), tw_of<T>(md, 0), tw_of<T>(md, 1), blk, V2, m1y, m2, s);
    mark(3);
    mark(4);
    blocked_view(4);
    mark(5);
  } else {
    fft_pass_strided(gz, g2, md.plan[1], Ny, Py, F * Nx, Pz, m1y, m2, false, tw_of<T>(md, 1),
                     md.y_row[prec], s);
    mark(3);
    blocked_view(3);
    if (stop <= 3) return;
    fft_mid_pass(g2, md.plan[0], Nx, (int)F, Py, Pz, md.H[0], md.H[1], md.H[2], ghat_of<T>(md),
                 tw_of<T>(md, 0), blk, V2, md.x_row[prec], s);
    mark(4);
    blocked_view(4);
    if (stop <= 4) return;
    fft_pass_strided(g2, g1, md.plan[1], Py, Ny, F * Nx, Pz, m2, m1y, true, tw_of<T>(md, 1),
                     md.y_row[prec], s);
    mark(5);
  }
  view(5, g1, (int64_t)Nx * Ny, Pz, (int64_t)Nx * Ny * Pzs, Pzs, 1);
  if (stop <= 5) return;
  if (full3d) {  // inspection: every line
    fft_pass_contig(g1, g0, md.plan[2], Pz, Nz, F * Nx * Ny, fftk::contig_map(Pzs),
                    fftk::contig_map(Nz), true, tw_of<T>(md, 2), s);
  } else {  // the lines the interpolation reads
    // into the field-interleaved grid [Nx][Ny][Nz][F]: the four fields of a
    // right-hand side at a stencil node are one 32-byte (c64) read
    const int64_t nl = md.n_occ_lines;
    fft_pass_contig(g1, g0, md.plan[2], Pz, Nz, F * nl,
                    fftk::fields_inner(F, V1, Pzs, 1, md.occ_lines, nl),
                    fftk::fields_inner(F, 1, (int64_t)Nz * F, F, md.occ_lines, nl, md.occ_zrange),
                    true, tw_of<T>(md, 2), s);
    view(6, g0, (int64_t)Nx * Ny, Nz, 1, (int64_t)Nz * F, F);
  }
  mark(6);
}

template <typename T, typename TX, typename TY>
void matvec_mesh(Plan *pl, MeshDev &md, int nrhs, const cx<TX> *x, int64_t ldx, cx<TY> *y,
                 int64_t ldy, hipStream_t s, hipEvent_t *ev) {
  const HostPlan &h = md.hp;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  far_stages<T, TX>(pl, md, nrhs, x, ldx, 6, s, ev);
  const cx<T> *phi = (const cx<T> *)pl->work[md.lane][prec][0];
  const bool plane = md.planar_z >= 0;  // fields on the scatterer's grid plane only
  const int64_t nf = 4 * (int64_t)nrhs;  // fields per node of the interleaved grid
  const int rows_per_block = 8;
  const int64_t blocks = (h.n + rows_per_block - 1) / rows_per_block;
  // right-hand sides per grid row: 4 or 2 when they divide nrhs
  const int rb = nrhs % 4 == 0 ? 4 : (nrhs % 2 == 0 ? 2 : 1);
  const bool cf = h.cfie;
  if (cf && (plane || !curl_of<T>(md))) throw Error(AIM_ERR_STATE, "combined field without curl weights");
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks, nrhs / rb), dim3(32 * rows_per_block), 0, s,
                       phi, nf, nrhs, plane ? plane_lam_of<T>(md) : lam_of<T>(md),
                       cf ? curl_of<T>(md) : nullptr, plane ? md.plane_anchor : md.anchor_lin,
                       plane ? md.plane_soff : md.stencil_off, plane ? md.plane_K : h.K,
                       md.rowptr, md.cols, near_of<T>(md), x, ldx, y, ldy, h.n,
                       (T)(h.alpha * h.k * kEta0), (T)(1.0 / (h.k * h.k)),
                       (T)((1.0 - h.alpha) * kEta0));
  };
  if (cf) {
    if (rb == 4)
      launch(k_interp_near<T, TX, TY, 4, true>);
    else if (rb == 2)
      launch(k_interp_near<T, TX, TY, 2, true>);
    else
      launch(k_interp_near<T, TX, TY, 1, true>);
  } else if (rb == 4) {
    launch(k_interp_near<T, TX, TY, 4, false>);
  } else if (rb == 2) {
    launch(k_interp_near<T, TX, TY, 2, false>);
  } else {
    launch(k_interp_near<T, TX, TY, 1, false>);
  }
  LAUNCHCHECK();
  if (ev) HIPCHECK(hipEventRecord(ev[7], s));
}

void assign_lanes(Plan *pl, const std::vector<double> &cost) {
  const int K = std::min(pl->nmesh, kMaxLanes);
  pl->nlanes = K;
  if (K > 1) {
    HIPCHECK(hipEventCreateWithFlags(&pl->lane_fork, hipEventDisableTiming));
    for (int l = 1; l < K; ++l) {
      HIPCHECK(hipStreamCreateWithFlags(&pl->lane_stream[l], hipStreamNonBlocking));
      HIPCHECK(hipEventCreateWithFlags(&pl->lane_join[l], hipEventDisableTiming));
    }
  }
  std::vector<int> order(pl->nmesh);
  for (int i = 0; i < pl->nmesh; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(K, 0.0);
  for (int i : order) {
    int l = 0;
    for (int j = 1; j < K; ++j)
      if (load[j] < load[l]) l = j;
    pl->mesh[i].lane = l;
    load[l] += cost[i];
  }
}

void release_lanes(Plan *pl) {
  for (int l = 1; l < kMaxLanes; ++l) {
    if (pl->lane_stream[l]) {
      (void)hipStreamSynchronize(pl->lane_stream[l]);
      (void)hipStreamDestroy(pl->lane_stream[l]);
    }
    if (pl->lane_join[l]) (void)hipEventDestroy(pl->lane_join[l]);
    pl->lane_stream[l] = nullptr;
    pl->lane_join[l] = nullptr;
  }
  if (pl->lane_fork) (void)hipEventDestroy(pl->lane_fork);
  pl->lane_fork = nullptr;
  pl->nlanes = 1;
}

void matvec_plan(Plan *pl, aim_precision prec, int nrhs, const void *x, void *y, hipStream_t s,
                 hipEvent_t *ev, const std::vector<char> *mesh_on) {
  const int64_t ld = pl->n_total;
  const bool lanes = pl->nlanes > 1 && !ev;
  if (lanes) {
    HIPCHECK(hipEventRecord(pl->lane_fork, s));
    for (int l = 1; l < pl->nlanes; ++l) HIPCHECK(hipStreamWaitEvent(pl->lane_stream[l], pl->lane_fork, 0));
  }
  int mi = 0;
  for (auto &md : pl->mesh) {
    if (mesh_on && !(*mesh_on)[mi]) {
      ++mi;
      continue;
    }
    const hipStream_t st = (lanes && md.lane > 0) ? pl->lane_stream[md.lane] : s;
    hipEvent_t *e = ev ? ev + (size_t)mi * (AIM_NSTAGE + 1) : nullptr;
    if (prec == AIM_FP64)
      matvec_mesh<double, double, double>(pl, md, nrhs, (const double2 *)x + md.offset, ld,
                                          (double2 *)y + md.offset, ld, st, e);
    else if (prec == AIM_MIXED)
      matvec_mesh<float, float, float>(pl, md, nrhs, (const float2 *)x + md.offset, ld,
                                       (float2 *)y + md.offset, ld, st, e);
    else
      matvec_mesh<float, double, double>(pl, md, nrhs, (const double2 *)x + md.offset, ld,
                                         (double2 *)y + md.offset, ld, st, e);
    ++mi;
  }
  if (lanes)
    for (int l = 1; l < pl->nlanes; ++l) {
      HIPCHECK(hipEventRecord(pl->lane_join[l], pl->lane_stream[l]));
      HIPCHECK(hipStreamWaitEvent(s, pl->lane_join[l], 0));
    }
}

template <typename T>
void copy_far_stage(Plan *pl, MeshDev &md, int nrhs, int stage, void *out, hipStream_t s) {
  const HostPlan &h = md.hp;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int Nx = h.grid[0], Ny = h.grid[1], Nz = h.grid[2];
  const int Py = h.pad[1], Pz = h.pad[2];
  const int64_t F = 4 * (int64_t)nrhs;
  const int blk = kGridBlock<T>;
  const int64_t V2 = (int64_t)Nx * Py * ((Pz + blk - 1) / blk * blk);
  if (thin_layout<T>(Pz) && stage >= 2 && stage <= 5) {  // [F][Pz][A] -> [F][A][Pz]
    const int64_t A = (stage == 3 || stage == 4) ? (int64_t)Nx * Py : (int64_t)Nx * Ny;
    const int64_t tot = F * A * Pz;
    hipLaunchKernelGGL((k_kz_inner<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       (const cx<T> *)pl->work[md.lane][prec][(stage == 3 || stage == 4) ? 2 : 1],
                       (cx<T> *)out, F, A, Pz);
    LAUNCHCHECK();
    return;
  }
  if (stage == 3 || stage == 4) {
    const int64_t tot = F * Nx * Py * Pz;
    hipLaunchKernelGGL((k_unblock<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       (const cx<T> *)pl->work[md.lane][prec][2], (cx<T> *)out, F, Nx, Py, Pz, blk, V2);
    LAUNCHCHECK();
    return;
  }
  if (stage == 2 || stage == 5) {  // drop the row padding
    const int Pzs = (Pz + blk - 1) / blk * blk;
    HIPCHECK(hipMemcpy2DAsync(out, sizeof(cx<T>) * Pz, pl->work[md.lane][prec][1], sizeof(cx<T>) * Pzs,
                              sizeof(cx<T>) * Pz, (size_t)(F * Nx * Ny), hipMemcpyDeviceToDevice, s));
    return;
  }
  // stage 1: the projected source grid; stage 6: the propagated fields
  HIPCHECK(hipMemcpyAsync(out, stage == 1 ? md.src[prec] : pl->work[md.lane][prec][0],
                          sizeof(cx<T>) * F * Nx * Ny * Nz, hipMemcpyDeviceToDevice, s));
}
template void copy_far_stage<double>(Plan *, MeshDev &, int, int, void *, hipStream_t);
template void copy_far_stage<float>(Plan *, MeshDev &, int, int, void *, hipStream_t);

namespace {
// out[(f A + a) Z + z] = in[f fs + a as + z zs] (inspection)
template <typename T>
__global__ void k_view_copy(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int64_t F,
                            int64_t A, int64_t Z, int64_t fs, int64_t as, int64_t zs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= F * A * Z) return;
  const int64_t z = t % Z, a = (t / Z) % A, f = t / (Z * A);
  out[t] = in[f * fs + a * as + z * zs];
}
}  // namespace

template <typename T>
void copy_stage_view(const StageView &v, void *out, hipStream_t s) {
  const int64_t tot = v.F * v.A * v.Z;
  const unsigned blocks = (unsigned)((tot + 255) / 256);
  if (v.kind == 1) {
    hipLaunchKernelGGL((k_view_copy<T>), dim3(blocks), dim3(256), 0, s, (const cx<T> *)v.p,
                       (cx<T> *)out, v.F, v.A, v.Z, v.fs, v.as, v.zs);
  } else if (v.kind == 2) {
    hipLaunchKernelGGL((k_unblock<T>), dim3(blocks), dim3(256), 0, s, (const cx<T> *)v.p,
                       (cx<T> *)out, v.F, v.Nx, v.Py, (int)v.Z, v.blk, v.fstride);
  } else {
    throw Error(AIM_ERR_ARG, "the product has no such stage for this mesh");
  }
  LAUNCHCHECK();
}
template void copy_stage_view<double>(const StageView &, void *, hipStream_t);
template void copy_stage_view<float>(const StageView &, void *, hipStream_t);

void autotune_mesh(Plan *pl, MeshDev &md, hipStream_t s) {
  const int64_t n = md.hp.n;
  // right-hand sides of the timed products (the caller's hint, else one)
  const int nr = std::max(1, (pl->params.tuning >> 16) & 0xff);
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  void *x = nullptr;
  try {
    x = dev_alloc(pl, sizeof(double2) * n * nr);
    HIPCHECK(hipMemsetAsync(x, 0, sizeof(double2) * n * nr, s));
    auto time_stages = [&](int prec, int stop) {
      for (int rep = 0; rep < 4; ++rep) {  // first repetition is a warm-up
        if (rep == 1) HIPCHECK(hipEventRecord(e0, s));
        if (prec == 0)
          far_stages<double, double>(pl, md, nr, (const double2 *)x, n, stop, s);
        else
          far_stages<float, double>(pl, md, nr, (const double2 *)x, n, stop, s);
      }
      HIPCHECK(hipEventRecord(e1, s));
      HIPCHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    // projection gather: occupied nodes per wave
    for (int prec = 0; prec < 2; ++prec) {
      if (prec == 1 && !pl->mixed) break;
      float best = 0;
      int choice = kGatherNpwCand[1];
      for (int c = 0; c < 3; ++c) {
        md.gather_npw[prec] = kGatherNpwCand[c];
        const float ms = time_stages(prec, 1);
        if (c == 0 || ms < best) {
          best = ms;
          choice = kGatherNpwCand[c];
        }
      }
      md.gather_npw[prec] = choice;
    }
    for (int prec = 0; prec < 2; ++prec) {
      if (prec == 1 && !pl->mixed) break;
      const bool thin = prec == 0 ? thin_layout<double>(md.hp.pad[2]) : thin_layout<float>(md.hp.pad[2]);
      if (thin || !fft_anterp_fused(md.plan[2])) {
        md.fuse_proj[prec] = 0;
        continue;
      }
      float best = 0;
      int choice = 0;
      for (int v = 0; v < 2; ++v) {
        md.fuse_proj[prec] = v;
        const float ms = time_stages(prec, 2);
        if (v == 0 || ms < best) {
          best = ms;
          choice = v;
        }
      }
      md.fuse_proj[prec] = choice;
    }
    // tile rows of the x pass and of the strided y passes (the whole far part
    // timed; 64-byte rows halve a work-group's LDS tile, so more work-groups
    // fit a CU, at the cost of half-cache-line accesses)
    for (int prec = 0; prec < 2; ++prec) {
      if (prec == 1 && !pl->mixed) break;
      const int forced = (pl->params.tuning >> 8) & 0xff;
      md.x_row[prec] = md.y_row[prec] = 128;
      if (forced == 1 || forced == 2) {  // 1: 128-byte rows, 2: 64-byte rows everywhere
        md.x_row[prec] = md.y_row[prec] = forced == 2 ? 64 : 128;
        continue;
      }
      // (a variant must beat 128-byte rows by 3%, the timing spread of
      // products of one right-hand side; by 1% where several are timed)
      const float margin = nr > 1 ? 0.99f : 0.97f;
      float best = 0, base = 0;
      int bx = 128, by = 128;
      for (int xr : {128, 64})
        for (int yr : {128, 64}) {
          md.x_row[prec] = xr;
          md.y_row[prec] = yr;
          const float ms = time_stages(prec, 6);
          if (xr == 128 && yr == 128) {
            best = base = ms;
          } else if (ms < best && ms < margin * base) {
            best = ms;
            bx = xr;
            by = yr;
          }
        }
      md.x_row[prec] = bx;
      md.y_row[prec] = by;
    }
    // field groups of the pipelined y / x / y passes (kz-blocked grids with
    // equal x and y lengths)
    for (int prec = 0; prec < 2; ++prec) {
      if (prec == 1 && !pl->mixed) break;
      md.xy_groups[prec] = 1;
      const bool thin = prec == 0 ? thin_layout<double>(md.hp.pad[2]) : thin_layout<float>(md.hp.pad[2]);
      if (thin || md.planar_z >= 0 || !xy_pipeline_available(md.plan[0], md.plan[1])) continue;
      const int forced = pl->params.tuning & 0xff;
      if (forced > 0) {
        md.xy_groups[prec] = forced;
        continue;
      }
      // the pipeline must beat the sequential passes by a clear margin: the
      // set-up times a few products of one right-hand side, and differences
      // of a few percent there are within run-to-run spread
      float best = 0, sequential = 0;
      int choice = 1;
      for (int g : {1, 2, 4}) {
        md.xy_groups[prec] = g;
        const float ms = time_stages(prec, 6);
        if (g == 1) {
          best = sequential = ms;
        } else if (ms < best && ms < 0.97f * sequential) {
          best = ms;
          choice = g;
        }
      }
      md.xy_groups[prec] = choice;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (x) dev_free(pl, x);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(pl, x);
}

template void far_stages<double, double>(Plan *, MeshDev &, int, const double2 *, int64_t, int,
                                         hipStream_t, hipEvent_t *, bool, StageView *);
template void far_stages<float, float>(Plan *, MeshDev &, int, const float2 *, int64_t, int,
                                       hipStream_t, hipEvent_t *, bool, StageView *);
template void far_stages<float, double>(Plan *, MeshDev &, int, const double2 *, int64_t, int,
                                        hipStream_t, hipEvent_t *, bool, StageView *);
template void matvec_mesh<double, double, double>(Plan *, MeshDev &, int, const double2 *, int64_t,
                                                  double2 *, int64_t, hipStream_t, hipEvent_t *);
template void matvec_mesh<float, float, float>(Plan *, MeshDev &, int, const float2 *, int64_t,
                                               float2 *, int64_t, hipStream_t, hipEvent_t *);
template void matvec_mesh<float, double, double>(Plan *, MeshDev &, int, const double2 *, int64_t,
                                                 double2 *, int64_t, hipStream_t, hipEvent_t *);

}  // namespace aim
