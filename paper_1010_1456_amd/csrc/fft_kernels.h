// Batched 1-D FFT passes over the AIM grid (forward/inverse, pruned).
//
// The propagation step convolves the projected sources with the grid Green's
// function on the doubled, zero-padded grid. Only the first N_d inputs of a
// forward line are non-zero and only the first N_d outputs of an inverse line
// are used (the pruning of the paper's Section 4.1 footnote), so every pass
// loads n_in <= P inputs and stores n_out <= P outputs per line.
//
// Each work-group processes a tile of lines; every thread owns at most one
// butterfly per Stockham stage and keeps its r values in registers; stages
// exchange through LDS. The stage radices are compile-time (one kernel set per
// FFT length, see fft_plans.h). Three pass shapes:
//  * contig  - lines contiguous along the transform (z lines),
//  * strided - transform along a strided axis, tile over contiguous lines
//              (y and x lines; consecutive lanes touch consecutive addresses),
//  * mid     - the x pass: forward FFT, multiply by the Green's spectrum
//              octant, inverse FFT, keeping each line in registers between the
//              last forward and the first inverse stage (inverse radices run in
//              reverse order, so the last forward butterfly's outputs are
//              exactly the first inverse butterfly's inputs).
#pragma once

#include <algorithm>

#include "aim_internal.h"
#include "fft_core.h"
#include "fft_map.h"
#include "fft_plans.h"

namespace aim {
namespace fftk {
using namespace fftc;

constexpr int kLdsBudget = 48 * 1024;


template <int R0, int R1, int R2>
struct PlanC {
  static constexpr int ns = (R1 == 1) ? 1 : ((R2 == 1) ? 2 : 3);
  static constexpr int P = R0 * R1 * R2;
  static constexpr int r(int s) { return s == 0 ? R0 : (s == 1 ? R1 : R2); }
  // product of the radices before stage s
  static constexpr int lb(int s) { return s == 0 ? 1 : (s == 1 ? R0 : R0 * R1); }
  // inverse plan: radices reversed
  static constexpr int ri(int s) { return r(ns - 1 - s); }
  static constexpr int lbi(int s) {
    int l = 1;
    for (int t = 0; t < s; ++t) l *= ri(t);
    return l;
  }
  static constexpr int maxnb() {
    int m = 0;
    for (int s = 0; s < ns; ++s) m = (P / r(s) > m) ? P / r(s) : m;
    return m;
  }
};

constexpr int round_up_c(int a, int b) { return (a + b - 1) / b * b; }

// Lines per work-group and threads per work-group of each pass shape.
template <typename T, class PC>
constexpr int tile_strided() {
  int B = sizeof(T) == 4 ? 16 : 8;  // 128-byte rows
  while (B > 1 && (PC::maxnb() * B > 1024 ||
                   (PC::ns > 1 && (long)PC::P * B * (long)sizeof(cx<T>) > kLdsBudget)))
    B /= 2;
  return B;
}
template <typename T, class PC>
constexpr int threads_strided() {
  return round_up_c(PC::maxnb() * tile_strided<T, PC>(), 64);
}
// x pass: lines per work-group (128-byte rows; 64- and 256-byte rows measured
// slower on the 324-point plan)
template <typename T, class PC>
constexpr int tile_mid() {
  return tile_strided<T, PC>();
}
template <typename T, class PC>
constexpr int threads_mid() {
  return round_up_c(PC::maxnb() * tile_mid<T, PC>(), 64);
}
template <typename T, class PC>
constexpr int tile_contig() {
  int B = 256 / PC::maxnb();
  if (B < 1) B = 1;
  const long line_bytes = (long)(PC::P + 1) * (long)sizeof(cx<T>);
  if (PC::ns > 1 && B * line_bytes > kLdsBudget) B = (int)(kLdsBudget / line_bytes);
  return B < 1 ? 1 : B;
}
template <typename T, class PC>
constexpr int threads_contig() {
  return round_up_c(PC::maxnb() * tile_contig<T, PC>(), 64);
}

template <typename T, bool INV, class PC>
__global__ void __launch_bounds__((threads_contig<T, PC>()))
    k_fft_contig(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int n_in, int n_out,
                 int64_t lines, int64_t in_ls, int64_t out_ls, const cx<T> *__restrict__ tw, int B) {
  using V = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  V *lds = reinterpret_cast<V *>(smem_raw);
  constexpr int P = PC::P, LS = P + 1;
  const int64_t line0 = (int64_t)blockIdx.x * B;
  V *twl = lds + (PC::ns > 1 ? B * LS : 0);  // twiddle table in LDS
  if constexpr (PC::ns > 1) {
    for (int i = threadIdx.x; i < P; i += blockDim.x) twl[i] = tw[i];
    __syncthreads();
  }
  static_for<PC::ns>([&](auto s_) AIM_AI {
    constexpr int s = decltype(s_)::value;
    constexpr int R = PC::r(s), L = PC::lb(s), Mp = P / (L * R), nb = P / R;
    constexpr bool first = (s == 0), last = (s == PC::ns - 1);
    const int b = threadIdx.x / nb, beta = threadIdx.x - b * nb;
    const bool active = (b < B) && (line0 + b < lines);
    const V *gin = in + (line0 + b) * in_ls;
    V *gout = out + (line0 + b) * out_ls;
    V *ll = lds + b * LS;
    (void)tw;
    auto ld = [&](int i) AIM_AI -> V {
      if constexpr (first) return (i < n_in) ? gin[i] : mk<V>((T)0, (T)0);
      else return ll[i];
    };
    auto st = [&](int i, V v) AIM_AI {
      if constexpr (last) {
        if (i < n_out) gout[i] = v;
      } else {
        ll[i] = v;
      }
    };
    V v[R];
    if (active) stage_load<R, INV, V>(v, beta, Mp, ld);
    if constexpr (!first && !last) __syncthreads();
    if (active) stage_compute_store<R, INV, V>(v, beta, L, Mp, twl, st);
    if constexpr (!last) __syncthreads();
  });
}

template <typename T, bool INV, class PC>
__global__ void __launch_bounds__((threads_strided<T, PC>()))
    k_fft_strided(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int n_in, int n_out,
                  int64_t inner, int ntile, LineMap imap, LineMap omap,
                  const cx<T> *__restrict__ tw, int) {
  using V = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  V *lds = reinterpret_cast<V *>(smem_raw);
  constexpr int P = PC::P;
  constexpr int B = tile_strided<T, PC>();
  const int64_t o = blockIdx.x / ntile;
  const int64_t c0 = (int64_t)(blockIdx.x % ntile) * B;
  const int b = threadIdx.x % B;
  const int beta = threadIdx.x / B;
  const bool line_ok = (c0 + b < inner);
  const V *gin = in + line_base(imap, o, c0 + b);
  V *gout = out + line_base(omap, o, c0 + b);
  // element offsets within a line fit in 32 bits (checked by the planner);
  // the first stage reads elements beta + q M' and the last writes
  // beta + p L, so address them from beta's element
  const int in_elem = (int)line_elem(imap), out_elem = (int)line_elem(omap);
  const V *gin_b = gin + beta * in_elem;
  V *gout_b = gout + beta * out_elem;
  V *twl = lds + (PC::ns > 1 ? P * B : 0);
  if constexpr (PC::ns > 1) {
    for (int i = threadIdx.x; i < P; i += blockDim.x) twl[i] = tw[i];
    __syncthreads();
  }
  static_for<PC::ns>([&](auto s_) AIM_AI {
    constexpr int s = decltype(s_)::value;
    constexpr int R = PC::r(s), L = PC::lb(s), Mp = P / (L * R), nb = P / R;
    constexpr bool first = (s == 0), last = (s == PC::ns - 1);
    const bool active = line_ok && (beta < nb);
    auto ld = [&](int i) AIM_AI -> V {
      if constexpr (first) return (i < n_in) ? gin_b[(i - beta) * in_elem] : mk<V>((T)0, (T)0);
      else return lds[i * B + b];
    };
    auto st = [&](int i, V v) AIM_AI {
      if constexpr (last) {
        if (i < n_out) gout_b[(i - beta) * out_elem] = v;
      } else {
        lds[i * B + b] = v;
      }
    };
    V v[R];
    if (active) stage_load<R, INV, V>(v, beta, Mp, ld);
    if constexpr (!first && !last) __syncthreads();
    if (active) stage_compute_store<R, INV, V>(v, beta, L, Mp, twl, st);
    if constexpr (!last) __syncthreads();
  });
}

// x pass over data in the kz-blocked layout [nfield][Pz/blk][n_x][Py][blk]
// (blk == 0: plain [nfield][n_x][Py][Pz]): lines (ky, kz), tile over kz. One
// work-group per (tile, field). Work-groups are dealt round-robin to the 8
// XCDs, so block ids are arranged for the fields of one tile to land on the
// same XCD back to back and share its L2 copy of the spectrum tile.
constexpr int kXcd = 8;

template <typename T, class PC>
__global__ void __launch_bounds__((threads_mid<T, PC>()))
    k_fft_mid(cx<T> *__restrict__ data, int n_x, int nfield, int Py, int Pz, int ntile, int Hy,
              int Hz, const cx<T> *__restrict__ ghat, const cx<T> *__restrict__ tw, int, int blk,
              int64_t fstride) {
  using V = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  V *lds = reinterpret_cast<V *>(smem_raw);
  constexpr int P = PC::P, ns = PC::ns;
  constexpr int B = tile_mid<T, PC>();
  const int xcd = blockIdx.x % kXcd;
  const int jb = blockIdx.x / kXcd;
  const int field = jb % nfield;
  const int tile = (jb / nfield) * kXcd + xcd;
  if (tile >= Py * ntile) return;  // padding blocks: exit before any barrier
  const int ky = tile / ntile;
  const int kz0 = (tile % ntile) * B;
  const int b = threadIdx.x % B;
  const int beta = threadIdx.x / B;
  const int kz = kz0 + b;
  const bool line_ok = kz < Pz;
  const int fky = (ky <= Py - ky) ? ky : Py - ky;
  const int fkz = (kz <= Pz - kz) ? kz : Pz - kz;
  const int gofs = fky * Hz + fkz;  // octant offsets fit in 32 bits
  const int gplane = Hy * Hz;
  const int es = blk == 0 ? Py * Pz : Py * blk;  // x stride (32-bit, checked by the planner)
  V *twl = lds + (ns > 1 ? P * B : 0);
  for (int i = threadIdx.x; i < P; i += blockDim.x) twl[i] = tw[i];
  __syncthreads();
  const int64_t lofs = blk == 0 ? (int64_t)ky * Pz + kz
                                : (int64_t)(kz / blk) * n_x * es + (int64_t)ky * blk + kz % blk;

  {
    V *line = data + field * fstride + lofs;
    V *line_b = line + beta * es;  // element beta of the line
    // forward stages except the last
    static_for<ns - 1>([&](auto s_) AIM_AI {
      constexpr int s = decltype(s_)::value;
      constexpr int R = PC::r(s), L = PC::lb(s), Mp = P / (L * R), nb = P / R;
      constexpr bool first = (s == 0);
      const bool active = line_ok && (beta < nb);
      auto ld = [&](int i) AIM_AI -> V {
        if constexpr (first) return (i < n_x) ? line_b[(i - beta) * es] : mk<V>((T)0, (T)0);
        else return lds[i * B + b];
      };
      auto st = [&](int i, V v) AIM_AI { lds[i * B + b] = v; };
      V v[R];
      if (active) stage_load<R, false, V>(v, beta, Mp, ld);
      if constexpr (!first) __syncthreads();
      if (active) stage_compute_store<R, false, V>(v, beta, L, Mp, twl, st);
      __syncthreads();
    });
    // last forward stage, spectrum multiply, first inverse stage in registers
    {
      constexpr int R = PC::r(ns - 1);
      constexpr int L = P / R;
      constexpr bool single = (ns == 1);
      const bool active = line_ok && (beta < L);
      const int j = beta;
      V v[R];
      if (active) {
        static_for<R>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          const int i = j * R + q;
          if constexpr (single) v[q] = (i < n_x) ? line[i * es] : mk<V>((T)0, (T)0);
          else v[q] = lds[i * B + b];
        });
      }
      if constexpr (!single) __syncthreads();
      if (active) {
        if constexpr (L > 1) {
          static_for<R - 1>([&](auto q_) AIM_AI {
            constexpr int q = decltype(q_)::value + 1;
            v[q] = tw_mul<false>(v[q], twl, j * q);
          });
        }
        Dft<R, false, V>::run(v);
        static_for<R>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value;
          const int kx = j + L * p;
          const int fkx = (kx <= P - kx) ? kx : P - kx;
          v[p] = cmul(v[p], ghat[fkx * gplane + gofs]);
        });
        Dft<R, true, V>::run(v);
        static_for<R>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value;
          const int i = p * L + j;
          if constexpr (single) {
            if (i < n_x) line[i * es] = v[p];
          } else {
            lds[i * B + b] = v[p];
          }
        });
      }
    }
    if constexpr (ns > 1) {
      __syncthreads();
      // remaining inverse stages, radices in reverse order
      static_for<ns - 1>([&](auto s_) AIM_AI {
        constexpr int s = decltype(s_)::value + 1;
        constexpr int R = PC::ri(s), L = PC::lbi(s), Mp = P / (L * R), nb = P / R;
        constexpr bool last = (s == ns - 1);
        const bool active = line_ok && (beta < nb);
        auto ld = [&](int i) AIM_AI -> V { return lds[i * B + b]; };
        auto st = [&](int i, V v) AIM_AI {
          if constexpr (last) {
            if (i < n_x) line_b[(i - beta) * es] = v;
          } else {
            lds[i * B + b] = v;
          }
        };
        V v[R];
        if (active) stage_load<R, true, V>(v, beta, Mp, ld);
        if constexpr (!last) __syncthreads();
        if (active) stage_compute_store<R, true, V>(v, beta, L, Mp, twl, st);
        if constexpr (!last) __syncthreads();
      });
    }
  }
}

template <typename T, class PC>
void launch_contig(const cx<T> *in, cx<T> *out, int n_in, int n_out, int64_t lines, int64_t in_ls,
                   int64_t out_ls, bool inverse, const cx<T> *tw, hipStream_t s) {
  constexpr int B = tile_contig<T, PC>();
  constexpr int threads = threads_contig<T, PC>();
  const size_t lds = PC::ns > 1 ? ((size_t)B * (PC::P + 1) + PC::P) * sizeof(cx<T>) : 0;
  const int64_t blocks = (lines + B - 1) / B;
  if (inverse)
    hipLaunchKernelGGL((k_fft_contig<T, true, PC>), dim3((unsigned)blocks), dim3(threads), lds, s,
                       in, out, n_in, n_out, lines, in_ls, out_ls, tw, B);
  else
    hipLaunchKernelGGL((k_fft_contig<T, false, PC>), dim3((unsigned)blocks), dim3(threads), lds, s,
                       in, out, n_in, n_out, lines, in_ls, out_ls, tw, B);
  LAUNCHCHECK();
}

template <typename T, class PC>
void launch_strided(const cx<T> *in, cx<T> *out, int n_in, int n_out, int64_t outer, int64_t inner,
                    const LineMap &imap, const LineMap &omap, bool inverse, const cx<T> *tw,
                    hipStream_t s) {
  constexpr int B = tile_strided<T, PC>();
  constexpr int threads = threads_strided<T, PC>();
  const int ntile = (int)((inner + B - 1) / B);
  const size_t lds = PC::ns > 1 ? (size_t)PC::P * (B + 1) * sizeof(cx<T>) : 0;
  const int64_t blocks = outer * ntile;
  if (inverse)
    hipLaunchKernelGGL((k_fft_strided<T, true, PC>), dim3((unsigned)blocks), dim3(threads), lds, s,
                       in, out, n_in, n_out, inner, ntile, imap, omap, tw, B);
  else
    hipLaunchKernelGGL((k_fft_strided<T, false, PC>), dim3((unsigned)blocks), dim3(threads), lds, s,
                       in, out, n_in, n_out, inner, ntile, imap, omap, tw, B);
  LAUNCHCHECK();
}

template <typename T, class PC>
void launch_mid(cx<T> *data, int n_x, int nfield, int Py, int Pz, int Hy, int Hz,
                const cx<T> *ghat, const cx<T> *tw, int blk, int64_t fstride, hipStream_t s) {
  constexpr int B = tile_mid<T, PC>();
  constexpr int threads = threads_mid<T, PC>();
  const int ntile = (Pz + B - 1) / B;
  const size_t lds = (size_t)PC::P * ((PC::ns > 1 ? B : 0) + 1) * sizeof(cx<T>);
  const int64_t tiles = ((int64_t)Py * ntile + kXcd - 1) / kXcd * kXcd;
  const int64_t blocks = tiles * nfield;
  hipLaunchKernelGGL((k_fft_mid<T, PC>), dim3((unsigned)blocks), dim3(threads), lds, s, data, n_x,
                     nfield, Py, Pz, ntile, Hy, Hz, ghat, tw, B, blk, fstride);
  LAUNCHCHECK();
}

[[noreturn]] inline void bad_length(int P) {
  throw Error(AIM_ERR_ARG, "no FFT kernels for length " + std::to_string(P));
}

}  // namespace fftk

}  // namespace aim
