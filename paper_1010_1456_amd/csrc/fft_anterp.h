// Anterpolation fused with the forward z pass.
//
// A work-group owns LB consecutive z lines (x, y) of the grid and, per right-
// hand side, (1) gathers the projected sources of the 4 fields on those lines
// into LDS from the node-ordered projection (entries of consecutive nodes are
// contiguous, so each wave loads 64 entries at a time, forms their products
// and every lane sums its own node's entries in a fixed order: bitwise
// reproducible, no atomics), then (2) runs the pruned forward z transform of
// the 4 x LB lines out of LDS and writes the P_z outputs of each line. The
// projected source grid is never written to memory.
#pragma once

#include "fft_kernels.h"

namespace aim {
namespace fftk {

template <typename T, class PC>
constexpr int anterp_lines() {
  // LB lines x 4 fields; keep the field buffer within the LDS budget
  int lb = 256 / (4 * PC::maxnb());
  if (lb < 1) lb = 1;
  const long per_line = 4L * (PC::P + 1) * (long)sizeof(cx<T>);
  while (lb > 1 && lb * per_line > kLdsBudget) --lb;
  return lb;
}
template <class PC>
constexpr bool anterp_fits() {  // every butterfly of 4 lines in one work-group
  return 4 * PC::maxnb() <= 1024;
}
template <typename T, class PC>
constexpr int anterp_threads() {
  const int t = round_up_c(4 * anterp_lines<T, PC>() * PC::maxnb(), 64);
  return t < 256 ? 256 : (t > 1024 ? 1024 : t);
}

// PR: at most P/2 grid nodes per line, so the first stage runs the
// upper-half-zero DFT (even first radix)
template <typename T, typename TX, bool PR, class PC>
__global__ void __launch_bounds__((anterp_threads<T, PC>()))
    k_anterp_fftz(const cx<TX> *__restrict__ x, int64_t ldx, int nrhs,
                  const int32_t *__restrict__ node_ptr, const int32_t *__restrict__ ent_col,
                  const T *__restrict__ lamT, int Nz, int64_t nlines, cx<T> *__restrict__ out,
                  int64_t out_ls, int64_t out_fstride, const cx<T> *__restrict__ tw) {
  using V = cx<T>;
  constexpr int P = PC::P, LS = P + 1;
  constexpr int LB = anterp_lines<T, PC>();
  constexpr int NW = anterp_threads<T, PC>() / 64;
  extern __shared__ unsigned char smem_raw[];
  V *buf = reinterpret_cast<V *>(smem_raw);            // [4 LB][LS]: field q, line l at (q LB + l)
  V *twl = buf + 4 * LB * LS;                          // [P]
  V *slot = twl + P;                                   // [NW][64][4]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t l0 = (int64_t)blockIdx.x * LB;
  const int nl = (int)((nlines - l0 < LB) ? nlines - l0 : LB);
  const int64_t node0 = l0 * Nz;
  const int nodes = nl * Nz;
  for (int i = threadIdx.x; i < P; i += blockDim.x) twl[i] = tw[i];

  for (int r = 0; r < nrhs; ++r) {
    const cx<TX> *xr = x + (int64_t)r * ldx;
    __syncthreads();  // buf free (previous right-hand side done), twl ready
    // ---- gather the 4 source fields of the block's lines into buf
    for (int c = wv * 64; c < nodes; c += NW * 64) {
      const int k = c + lane;
      const bool ok = k < nodes;
      const int64_t v = node0 + k;
      const int e0 = ok ? node_ptr[v] : 0, e1 = ok ? node_ptr[v + 1] : 0;
      const int cend = (c + 64 < nodes) ? c + 64 : nodes;
      const int w0 = node_ptr[node0 + c], w1 = node_ptr[node0 + cend];
      T a[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      V *sl = slot + wv * 256;
      for (int c0 = w0; c0 < w1; c0 += 64) {
        const int e = c0 + lane;
        if (e < w1) {
          const cx<TX> xv = xr[ent_col[e]];
          const T xa = (T)xv.x, xb = (T)xv.y;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T wq = lamT[(int64_t)e * 4 + q];
            sl[lane * 4 + q] = mk<V>(wq * xa, wq * xb);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int lo = (e0 > c0 ? e0 : c0) - c0, hi = (e1 < c0 + 64 ? e1 : c0 + 64) - c0;
        for (int kk = lo; kk < hi; ++kk) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const V p = sl[kk * 4 + q];
            a[q][0] += p.x;
            a[q][1] += p.y;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      if (ok) {
        const int l = k / Nz, z = k - l * Nz;
#pragma unroll
        for (int q = 0; q < 4; ++q) buf[(q * LB + l) * LS + z] = mk<V>(a[q][0], a[q][1]);
      }
    }
    __syncthreads();
    // ---- pruned forward z transform of the 4 LB lines, in place in buf
    static_for<PC::ns>([&](auto s_) AIM_AI {
      constexpr int s = decltype(s_)::value;
      constexpr int R = PC::r(s), L = PC::lb(s), Mp = P / (L * R), nb = P / R;
      constexpr bool first = (s == 0), last = (s == PC::ns - 1);
      const int bl = threadIdx.x / nb, beta = threadIdx.x - bl * nb;
      const int q = bl / LB, l = bl - q * LB;
      const bool active = (bl < 4 * LB) && (l < nl);
      V *ll = buf + bl * LS;
      V *gout = out + (int64_t)(r * 4 + q) * out_fstride + (l0 + l) * out_ls;
      auto ld = [&](int i) AIM_AI -> V {
        if constexpr (first) return (i < Nz) ? ll[i] : mk<V>((T)0, (T)0);
        else return ll[i];
      };
      auto st = [&](int i, V v) AIM_AI {
        if constexpr (last) gout[i] = v;
        else ll[i] = v;
      };
      constexpr bool uz = stage_uz<R, false, PR, first, last>();
      V v[R];
      if (active) {
        if constexpr (uz) stage_load_p<R, R / 2, V>(v, beta, Mp, ld);
        else stage_load<R, false, V>(v, beta, Mp, ld);
      }
      if constexpr (!last) __syncthreads();
      if (active) stage_compute_store_p<R, false, uz, R, false>(v, beta, L, Mp, twl, st);
      if constexpr (!last) __syncthreads();
    });
  }
}

// false if the length has no fused kernel (the caller then projects and
// transforms in two launches)
template <typename T, typename TX, class PC>
bool launch_anterp_fftz(const cx<TX> *x, int64_t ldx, int nrhs, const int32_t *node_ptr,
                        const int32_t *ent_col, const T *lamT, int Nz, int64_t nlines,
                        cx<T> *out, int64_t out_ls, int64_t out_fstride, const cx<T> *tw,
                        hipStream_t s) {
  if constexpr (!anterp_fits<PC>()) {
    return false;
  } else {
  constexpr int LB = anterp_lines<T, PC>();
  constexpr int threads = anterp_threads<T, PC>();
  const size_t lds = ((size_t)4 * LB * (PC::P + 1) + PC::P + (size_t)(threads / 64) * 256) *
                     sizeof(cx<T>);
  const int64_t blocks = (nlines + LB - 1) / LB;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), lds, s, x, ldx, nrhs, node_ptr,
                       ent_col, lamT, Nz, nlines, out, out_ls, out_fstride, tw);
  };
  if (pass_prunable<PC>(false, Nz, 0))
    go(k_anterp_fftz<T, TX, true, PC>);
  else
    go(k_anterp_fftz<T, TX, false, PC>);
  LAUNCHCHECK();
  return true;
  }
}

}  // namespace fftk
}  // namespace aim
