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
#include <type_traits>

#include "aim_internal.h"
#include "fft_core.h"
#include "fft_map.h"
#include "fft_plans.h"

namespace aim {
namespace fftk {
using namespace fftc;

constexpr int kLdsBudget = 48 * 1024;
// Work-groups of a launch are dealt round-robin to the 8 XCDs, each with its
// own L2; kernels that number their work in contiguous ranges per XCD
// (block b does item (b % kXcd) * slots + b / kXcd) keep neighbouring items,
// e.g. the fields of one grid line, in one L2.
constexpr int kXcd = 8;

using u32x2 = unsigned int __attribute__((ext_vector_type(2)));
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

// Passes over a grid larger than the 256 MB last-level cache load and store it
// non-temporally (the "nt" cache policy: each element is streamed through the
// caches once): the y passes, and the x pass in the kz-blocked layout.
// Measured on the 8-lambda sphere (541 MB per pass, c64): forward y 0.164 ->
// 0.150 ms, x pass 0.355 -> 0.325, inverse y 0.151 -> 0.138. Smaller grids
// keep the default policy, under which a pass can find its input still in that
// cache (the uneven batch, whose small members' grids fit: c64 product 2.365
// ms with the nt policy on every grid, 2.336 ms with it on the large ones
// only). The z passes always keep the default: their strided stores measured
// slower with the nt policy (8-lambda sphere, forward z 0.067 -> 0.099 ms).
constexpr uint64_t kStreamBytes = 256ull << 20;
template <bool NT, typename V>
__device__ __forceinline__ V stream_load(const V *p) {
  if constexpr (!NT)
    return *p;
  else if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p)));
  else
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p)));
}
template <bool NT, typename V>
__device__ __forceinline__ void stream_store(V *p, V v) {
  if constexpr (!NT)
    *p = v;
  else if constexpr (sizeof(V) == 8)
    __builtin_nontemporal_store(__builtin_bit_cast(u32x2, v), reinterpret_cast<u32x2 *>(p));
  else
    __builtin_nontemporal_store(__builtin_bit_cast(u32x4, v), reinterpret_cast<u32x4 *>(p));
}

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

// Lines per work-group and threads per work-group of each pass shape: a
// tile spans row_bytes of consecutive lines, fewer if the lines' butterflies
// or their LDS exchange would not fit one work-group.
template <typename T, class PC>
constexpr int tile_rows(int row_bytes) {
  int B = row_bytes / (int)sizeof(cx<T>);
  while (B > 1 && (PC::maxnb() * B > 1024 ||
                   (PC::ns > 1 && (long)PC::P * B * (long)sizeof(cx<T>) > kLdsBudget)))
    B /= 2;
  return B;
}
// Strided (y) and x passes: a tile spans ROW bytes of consecutive lines, 128
// (one cache line) or 64; the set-up picks per mesh and precision by timing.
template <typename T, class PC, int ROW = 128>
constexpr int tile_strided() {
  return tile_rows<T, PC>(ROW);
}
template <typename T, class PC, int ROW = 128>
constexpr int threads_strided() {
  return round_up_c(PC::maxnb() * tile_strided<T, PC, ROW>(), 64);
}
template <typename T, class PC, int ROW = 128>
constexpr int tile_mid() {
  return tile_rows<T, PC>(ROW);
}
// Wide x-pass work-groups, for two-stage plans whose first radix is twice the
// middle one (P = 2 R R, e.g. 162 = 18 x 9): the first and last stages have
// half as many butterflies per line as the middle stage, so with one thread
// per middle butterfly half the threads idle in those stages. A wide
// work-group gives each line R threads instead, each thread two middle
// butterflies, and takes kMidWideRows rows (tiles) of lines, so that the
// thread count fills whole waves.
constexpr int kMidWideRows = 4;
template <class PC>
constexpr bool mid_wide_plan() {
  return PC::ns == 2 && PC::r(0) == 2 * PC::r(1);
}
// threads per line of an x-pass work-group
template <class PC, bool WIDE>
constexpr int mid_tpl() {
  return WIDE ? PC::P / PC::r(0) : PC::maxnb();
}
template <typename T, class PC, int ROW = 128, bool WIDE = false>
constexpr int threads_mid() {
  return round_up_c(mid_tpl<PC, WIDE>() * tile_mid<T, PC, ROW>() * (WIDE ? kMidWideRows : 1), 64);
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

// PR (pruned): a forward pass whose lines hold at most P/2 inputs runs its
// first stage as the upper-half-zero DFT; an inverse pass that keeps at most
// P/2 outputs computes only the lower half of its last stage's outputs (both
// need an even radix there).
template <int R, bool INV, bool PR, bool FIRST, bool LAST>
constexpr bool stage_uz() {
  return PR && !INV && FIRST && R % 2 == 0;
}
template <int R, bool INV, bool PR, bool FIRST, bool LAST>
constexpr int stage_nout() {
  return (PR && INV && LAST && R % 2 == 0) ? R / 2 : R;
}
template <class PC>
bool pass_prunable(bool inverse, int n_in, int n_out) {
  return inverse ? (PC::r(PC::ns - 1) % 2 == 0 && 2 * n_out <= PC::P)
                 : (PC::r(0) % 2 == 0 && 2 * n_in <= PC::P);
}

template <typename T, bool INV, bool PR, class PC>
__global__ void __launch_bounds__((threads_contig<T, PC>()))
    k_fft_contig(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int n_in, int n_out,
                 int64_t lines, ContigMap imap, ContigMap omap, const cx<T> *__restrict__ tw,
                 int B, int64_t slots) {
  using V = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  V *lds = reinterpret_cast<V *>(smem_raw);
  constexpr int P = PC::P, LS = P + 1;
  // slots > 0: tiles in contiguous ranges per XCD, so that the fields of a
  // line (consecutive pass lines of an interleaved layout) that fall in
  // different tiles go through one L2; tiles past the last line have no
  // active thread
  const int64_t tile =
      slots ? (int64_t)(blockIdx.x % kXcd) * slots + blockIdx.x / kXcd : (int64_t)blockIdx.x;
  const int64_t line0 = tile * B;
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
    // threads past the last line address the last line (the line selection
    // and range tables are read for every thread; nothing is loaded or
    // stored for them)
    const int64_t Lc = active ? line0 + b : lines - 1;
    // line bases only where the stage touches global memory; element offsets
    // within a line fit 32 bits (checked by the launcher)
    const V *gin = nullptr;
    V *gout = nullptr;
    if constexpr (first) gin = in + contig_base(imap, Lc);
    if constexpr (last) gout = out + contig_base(omap, Lc);
    const int es_in = (int)imap.es, es_out = (int)omap.es;
    V *ll = lds + b * LS;
    (void)tw;
    // element ranges [lo, g0) and [g1, hi) of the line (all of it without a
    // range table): a line through a closed surface holds sources where it
    // crosses the surface, and none in the gap between. Inputs are read over
    // [lo, hi) (zeros in the gap; skipping its reads measured slower for
    // c128), outputs stored outside the gap only.
    int in_lo = 0, in_hi = n_in;
    int out_lo = 0, out_g0 = n_out, out_g1 = n_out, out_hi = n_out;
    if (first && imap.range) {
      const int32_t *rg = imap.range + 4 * sel_index(imap, Lc);
      in_lo = rg[0];
      in_hi = min(n_in, rg[3]);
    }
    if (last && omap.range) {
      const int32_t *rg = omap.range + 4 * sel_index(omap, Lc);
      out_lo = rg[0];
      out_g0 = rg[1];
      out_g1 = rg[2];
      out_hi = min(n_out, rg[3]);
    }
    auto ld = [&](int i) AIM_AI -> V {
      if constexpr (first)
        return (i >= in_lo && i < in_hi) ? gin[i * es_in] : mk<V>((T)0, (T)0);
      else return ll[i];
    };
    auto st = [&](int i, V v) AIM_AI {
      if constexpr (last) {
        if (i >= out_lo && i < out_hi && (i < out_g0 || i >= out_g1)) gout[i * es_out] = v;
      } else {
        ll[i] = v;
      }
    };
    constexpr bool uz = stage_uz<R, INV, PR, first, last>();
    constexpr int nout = stage_nout<R, INV, PR, first, last>();
    V v[R];
    if (active) {
      if constexpr (uz) stage_load_p<R, R / 2, V>(v, beta, Mp, ld);
      else stage_load<R, INV, V>(v, beta, Mp, ld);
    }
    if constexpr (!first && !last) __syncthreads();
    if (active) stage_compute_store_p<R, INV, uz, nout, false>(v, beta, L, Mp, twl, st);
    if constexpr (!last) __syncthreads();
  });
}

// One work-group of a strided pass: tile vb = o ntile + (c0 / B) covers the
// B lines (o, c0 .. c0 + B - 1).
template <typename T, bool INV, bool PR, class PC, int ROW = 128, bool NT = true>
__device__ __forceinline__ void strided_body(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                             int n_in, int n_out, int64_t inner, int ntile,
                                             const LineMap &imap, const LineMap &omap,
                                             const cx<T> *__restrict__ tw, int64_t vb) {
  using V = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  V *lds = reinterpret_cast<V *>(smem_raw);
  constexpr int P = PC::P;
  constexpr int B = tile_strided<T, PC, ROW>();
  const int vt = (int)vb;  // < 2^31 (launch size)
  const int o = vt / ntile;
  const int c0 = (vt - o * ntile) * B;
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
  // element ranges of this line (all of it without a range table)
  int in_lo = 0, in_hi = n_in, out_lo = 0, out_hi = n_out;
  if (imap.range) {
    const int r = o % imap.range_rows;
    in_lo = imap.range[2 * r];
    in_hi = min(n_in, imap.range[2 * r + 1]);
  }
  if (omap.range) {
    const int r = o % omap.range_rows;
    out_lo = omap.range[2 * r];
    out_hi = min(n_out, omap.range[2 * r + 1]);
  }
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
      if constexpr (first)
        return (i >= in_lo && i < in_hi) ? stream_load<NT>(&gin_b[(i - beta) * in_elem])
                                         : mk<V>((T)0, (T)0);
      else return lds[i * B + b];
    };
    auto st = [&](int i, V v) AIM_AI {
      if constexpr (last) {
        if (i >= out_lo && i < out_hi) stream_store<NT>(&gout_b[(i - beta) * out_elem], v);
      } else {
        lds[i * B + b] = v;
      }
    };
    constexpr bool uz = stage_uz<R, INV, PR, first, last>();
    constexpr int nout = stage_nout<R, INV, PR, first, last>();
    V v[R];
    if (active) {
      if constexpr (uz) stage_load_p<R, R / 2, V>(v, beta, Mp, ld);
      else stage_load<R, INV, V>(v, beta, Mp, ld);
    }
    if constexpr (!first && !last) __syncthreads();
    if (active) stage_compute_store_p<R, INV, uz, nout, false>(v, beta, L, Mp, twl, st);
    if constexpr (!last) __syncthreads();
  });
}

template <typename T, bool INV, bool PR, class PC, int ROW, bool NT>
__global__ void __launch_bounds__((threads_strided<T, PC, ROW>()))
    k_fft_strided(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int n_in, int n_out,
                  int64_t inner, int ntile, LineMap imap, LineMap omap,
                  const cx<T> *__restrict__ tw, int64_t tiles, int64_t slots) {
  int64_t vb = blockIdx.x;
  if constexpr (ROW < 128) {
    // two tiles share each 128-byte line: adjacent tiles go to one XCD (its
    // tiles in one contiguous range, taken in order), so the second read of a
    // line, and the second half of a line's writes, meet the first in its L2
    vb = (int64_t)(blockIdx.x % kXcd) * slots + blockIdx.x / kXcd;
    if (vb >= tiles) return;  // the whole work-group
  }
  strided_body<T, INV, PR, PC, ROW, NT>(in, out, n_in, n_out, inner, ntile, imap, omap, tw, vb);
}

// x pass: forward transform along x, spectrum multiply and inverse transform
// of every line (ky, kz) of every field. A work-group owns a tile of B lines
// that are adjacent in memory (one 128-byte row: consecutive kz of the
// kz-blocked layout, or consecutive ky of the thin layout) in one field. The
// fields of a tile, and the fields of its mirror tile (Py - ky, resp.
// Pz - kz: the same octant rows), get consecutive numbers, and consecutive
// numbers go to the same XCD, so the octant rows a tile reads are mostly
// found in that XCD's L2.
// Global accesses are buffer loads and stores: a work-group-uniform resource
// and scalar offset plus a per-thread 32-bit offset fixed for the whole kernel
// (the launcher checks the ranges), which keeps address arithmetic off the
// vector ALU.
constexpr int kBufferWord3 = 0x00020000;  // raw buffer resource, 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           kBufferWord3);
}
template <typename V, int AUX = 0>
__device__ __forceinline__ V bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V,
                              __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
  else
    return __builtin_bit_cast(V,
                              __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, AUX));
}
template <typename V, int AUX = 0>
__device__ __forceinline__ void bstore(V v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       uint32_t soff) {
  if constexpr (sizeof(V) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff,
                                          AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)voff, (int)soff,
                                           AUX);
}

// waves per SIMD the x pass aims to fit in registers where LDS allows them
template <typename T>
constexpr int mid_target_waves() {
  return sizeof(T) == 4 ? 7 : 3;
}
// LDS of the x pass: the tile's lines, and for two-stage plans the row tables
// of the middle stage and of the inverse's last stage (about P entries), for
// three-stage plans the twiddle table of exp(-2 pi i e / P): row tables of
// long lines would cost about as much LDS as the lines themselves (measured on
// the 2592-point plan: 1.66 ms with row tables, 1.17 ms without)
// Where the tile's lines would limit the work-groups per CU below what the
// registers allow, two-stage plans exchange each line through LDS in two
// halves (the first ceil(R/2) outputs of every butterfly, then the rest), so
// the line buffer holds about half a tile (8-lambda sphere, 324-point lines:
// 3 -> 5 work-groups per CU for c64, 0.357 -> 0.352 ms; 3 -> 6 for c128,
// 0.676 -> 0.629 ms). Shorter lines keep the one-step exchange: their tiles
// do not limit the occupancy, and the extra barriers cost time.
template <typename T, class PC, int ROW = 128, bool WIDE = false>
struct MidLds {
  static constexpr int P = PC::P, ns = PC::ns, R0 = PC::r(0), RM = PC::r(ns - 1);
  static constexpr bool rows = ns == 2;
  static constexpr int flat = ns > 2 ? P : 0;
  static constexpr int mid_rows = rows ? (P / RM) * (RM - 1) : 0;
  static constexpr bool same_rows = (R0 == RM);  // square two-stage plans share one table
  static constexpr int last_rows = (rows && !same_rows) ? (P / R0) * (R0 - 1) : 0;
  static constexpr int S0 = (R0 + 1) / 2, S1 = (RM + 1) / 2;  // first-half output counts
  static constexpr int half = (S0 * RM > S1 * R0 ? S0 * RM : S1 * R0);
  static constexpr int B = tile_mid<T, PC, ROW>() * (WIDE ? kMidWideRows : 1);  // lines
  static constexpr long tables = (long)(flat + mid_rows + last_rows) * (long)sizeof(cx<T>);
  static constexpr long lds_cu = 160 * 1024;
  static constexpr int groups_by_waves =
      4 * mid_target_waves<T>() / ((threads_mid<T, PC, ROW, WIDE>() + 63) / 64);
  static constexpr bool split =
      ns == 2 &&
      (WIDE || lds_cu / ((long)P * B * (long)sizeof(cx<T>) + tables) < groups_by_waves);
  static constexpr int data = ns > 1 ? (split ? half : P) * B : 0;
  static constexpr int total = data + flat + mid_rows + last_rows;
};
// waves per SIMD the x pass must fit in registers: the target where the split
// exchange or a three-stage plan leaves LDS for them (128-lambda plate,
// 2592-point lines: 0.173 -> 0.165 ms for c64), else 4 for c64 (shorter
// lines measured slower when squeezed to 72 registers)
template <typename T, class PC, int ROW = 128, bool WIDE = false>
constexpr int mid_min_waves() {
  return (sizeof(T) == 8 || MidLds<T, PC, ROW, WIDE>::split || PC::ns > 2) ? mid_target_waves<T>()
                                                                           : 4;
}

// One work-group of the x pass: vb is the launch's block number (XCD vb % 8).
template <typename T, class PC, bool KYL, int ROW = 128, bool WIDE = false, bool NT = true>
__device__ __forceinline__ void mid_body(cx<T> *__restrict__ data, int n_x, int nfield, int Py,
                                         int Pz, int ntile, int slots, int Hy, int Hz,
                                         const cx<T> *__restrict__ ghat,
                                         const cx<T> *__restrict__ tw, int64_t fstride,
                                         const FastDiv &dfield, const FastDiv &dtile,
                                         int64_t vb) {
  using V = cx<T>;
  using ML = MidLds<T, PC, ROW, WIDE>;
  extern __shared__ unsigned char smem_raw[];
  V *lds = reinterpret_cast<V *>(smem_raw);
  constexpr int P = PC::P, ns = PC::ns;
  constexpr int B = ML::B;  // lines of the work-group (consecutive along the tile axis)
  static_assert(!WIDE || (mid_wide_plan<PC>() && ML::split), "wide work-groups");
  constexpr uint32_t SV = sizeof(V);
  // NT: the lines are loaded and stored non-temporally (buffer cache policy
  // bit 1); the thin layout of the plates keeps the default policy
  // (128-lambda plate: x pass 0.165 -> 0.405 ms with the nt policy)
  constexpr int kNtAux = (NT && !KYL) ? 2 : 0;
  // a line holds at most P/2 sources (n_x <= P/2 for even P, checked by the
  // launcher) and only its first P/2 outputs are kept: with an even first
  // radix the forward transform's first stage skips the zero upper half of
  // its inputs and the inverse transform's last stage (same radix) computes
  // the lower half of its outputs only
  constexpr bool HALF = (PC::r(0) % 2 == 0);
  constexpr int R0 = PC::r(0), Mp0 = P / R0;      // first stage: L = 1, M' = nb = P / R0
  constexpr int NIN0 = HALF ? R0 / 2 : R0;        // first-stage inputs per butterfly
  constexpr int RM = PC::r(ns - 1), LM = P / RM;  // middle stage (M' = 1)

  // Lines run along x at (ky, kz). kz-blocked layout (KYL false): a tile is
  // B consecutive kz (the tile axis) at one ky (the fixed axis). Thin layout
  // [nfield][Pz][n_x][Py] (KYL true): B consecutive ky at one kz. Work number
  // t = nfield (2 (ff ntile + kt) + m) + field: fixed index ff (m = 0) or its
  // mirror Pf - ff (m = 1), which reads the same octant rows, tile kt.
  const int Pt = KYL ? Py : Pz, Pf = KYL ? Pz : Py;
  const int t = (int)(vb % kXcd) * slots + (int)(vb / kXcd);
  const int tt = (int)fast_div((uint32_t)t, dfield), field = t - tt * nfield;
  const int m = tt & 1, rest = tt >> 1;
  const int ff = (int)fast_div((uint32_t)rest, dtile);
  const int kt = rest - ff * ntile;
  if (2 * ff > Pf) return;                      // padding: exit before any barrier
  if (m && (ff == 0 || 2 * ff == Pf)) return;  // its own mirror: m = 0 covers it
  const int fixed = m ? Pf - ff : ff;
  const int k0 = kt * B;
  const int b = threadIdx.x % B;
  const int beta = threadIdx.x / B;
  const int kl = k0 + b;  // tile-axis index of this thread's line
  const bool line_ok = kl < Pt;
  const int fl = (kl <= Pt - kl) ? kl : Pt - kl;
  const int fky = KYL ? fl : ff, fkz = KYL ? ff : fl;
  const int gplane = Hy * Hz;
  // kz block of the kz-blocked layout: 128 bytes of consecutive kz (checked by
  // the launchers)
  constexpr int blk = kGridBlock<T>;
  const int es = KYL ? Py : Py * blk;  // elements between x and x + 1 of a line
  // field data: resource over the kz blocks of the work-group's lines (one kz
  // plane for KYL) of this field; its first line starts at byte t0, thread
  // (b, beta) adds o_beta
  const int64_t blk_elems = (int64_t)n_x * es;
  constexpr int WB = WIDE ? kMidWideRows : 1;  // kz blocks a work-group may span
  const int kb0 = KYL ? fixed : k0 / blk;
  const int nres = KYL ? 1 : min(WB, (Pz + blk - 1) / blk - kb0);
  const __amdgpu_buffer_rsrc_t fr = buffer_of(data + field * fstride + (int64_t)kb0 * blk_elems,
                                              (uint32_t)(blk_elems * nres) * SV);
  const int kin = KYL ? 0 : k0 % blk + b;  // the line's kz from its first block
  const uint32_t t0 = (uint32_t)(KYL ? k0 : fixed * blk) * SV;
  const uint32_t o_beta =
      (uint32_t)((KYL || !WIDE) ? (KYL ? b : kin) + beta * es
                                : (int64_t)(kin / blk) * blk_elems + kin % blk + (int64_t)beta * es) *
      SV;

  // spectrum values of the middle butterfly j = beta (kx = j + LM p): kx <
  // P/2 for 2p <= RM - 2 (row kx), kx >= P/2 for 2p >= RM (row P - kx); only
  // the middle p of an odd RM is folded at run time. Loaded where they are
  // used: issued at entry they delay the first stage's loads.
  const int j = beta;
  const bool act_mid = line_ok && (beta < LM);
  auto spectrum = [&](V *g, const int j) AIM_AI {
    const int gofs = fky * Hz + fkz;
    const __amdgpu_buffer_rsrc_t gres =
        buffer_of(ghat, (uint32_t)gplane * (uint32_t)(P / 2 + 1) * SV);
    const uint32_t g_lo = (uint32_t)(j * gplane + gofs) * SV;
    const uint32_t g_hi = (uint32_t)((LM - 1 - j) * gplane + gofs) * SV;
    static_for<RM>([&](auto p_) AIM_AI {
      constexpr int p = decltype(p_)::value;
      if constexpr (2 * p <= RM - 2) {
        g[p] = bload<V>(gres, g_lo, (uint32_t)(LM * p * gplane) * SV);
      } else if constexpr (2 * p >= RM) {
        g[p] = bload<V>(gres, g_hi, (uint32_t)((P - LM * p - LM + 1) * gplane) * SV);
      } else {
        const int kx = j + LM * p;
        const int fkx = (kx <= P - kx) ? kx : P - kx;
        g[p] = bload<V>(gres, (uint32_t)(fkx * gplane + gofs) * SV, 0u);
      }
    });
  };

  // first-stage inputs: butterfly beta reads elements beta + q M' (q < NIN0)
  const bool act0 = line_ok && (beta < Mp0);
  V v0[R0];
  if (act0)
    static_for<NIN0>([&](auto q_) AIM_AI {
      constexpr int q = decltype(q_)::value;
      v0[q] = (beta + q * Mp0 < n_x)
                  ? bload<V, kNtAux>(fr, o_beta, t0 + (uint32_t)(q * Mp0 * es) * SV)
                  : mk<V>((T)0, (T)0);
    });

  V *twl = lds + ML::data;                            // flat table (3-stage plans)
  V *twm = twl + ML::flat;                            // middle stage rows
  V *twr = ML::same_rows ? twm : twm + ML::mid_rows;  // inverse last stage rows
  if constexpr (ML::flat > 0)
    for (int i = threadIdx.x; i < P; i += blockDim.x) twl[i] = tw[i];
  if constexpr (ML::rows) {
    for (int i = threadIdx.x; i < ML::mid_rows; i += blockDim.x) {
      const int jj = i / (RM - 1), q = i - jj * (RM - 1) + 1;
      twm[i] = tw[jj * q];
    }
    if constexpr (!ML::same_rows)
      for (int i = threadIdx.x; i < ML::last_rows; i += blockDim.x) {
        const int jj = i / (R0 - 1), q = i - jj * (R0 - 1) + 1;
        twr[i] = tw[jj * q];
      }
  }

  if constexpr (ns == 1) {
    // one stage (L = 1, only beta = 0 works): forward DFT, multiply, inverse
    // DFT, all in registers
    if (act0) {
      if constexpr (HALF) dft_upper_zero<R0, false, V>(v0);
      else Dft<R0, false, V>::run(v0);
      V g[R0];
      spectrum(g, j);
      static_for<R0>([&](auto p_) AIM_AI {
        constexpr int p = decltype(p_)::value;
        v0[p] = cmul(v0[p], g[p]);
      });
      Dft<R0, true, V>::run(v0);
      static_for<NIN0>([&](auto p_) AIM_AI {
        constexpr int p = decltype(p_)::value;
        if (p < n_x) bstore<V, kNtAux>(v0[p], fr, o_beta, t0 + (uint32_t)(p * es) * SV);
      });
    }
  } else if constexpr (WIDE) {
    // P = R0 RM with R0 = 2 RM: thread beta < RM of a line runs first-stage
    // butterfly beta, middle butterflies beta and beta + RM, and last-stage
    // butterfly beta. Exchange 1 in two halves: first-stage outputs p < RM
    // feed middle butterflies j < RM (each thread's first), p >= RM the others;
    // exchange 2 by output halves as in the split exchange below.
    constexpr int S1 = ML::S1;
    const bool act = line_ok && (beta < RM);  // Mp0 = P / R0 = RM
    __syncthreads();  // twiddle tables ready
    if (act) dft_upper_zero<R0, false, V>(v0);
    V va[RM], vb[RM];
    static_for<2>([&](auto h_) AIM_AI {
      constexpr int h = decltype(h_)::value;
      // stage-1 output p (< R0) of butterfly beta is element p RM + beta;
      // middle butterfly jj reads elements jj RM + q
      if (act)
        static_for<RM>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value;
          lds[(p * RM + beta) * B + b] = v0[p + h * RM];
        });
      __syncthreads();
      if (act)
        static_for<RM>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          (h ? vb : va)[q] = lds[(beta * RM + q) * B + b];
        });
      __syncthreads();
    });
    auto middle = [&](V *v, const int jj) AIM_AI {
      const V *row = twm + jj * (RM - 1);
      static_for<RM - 1>([&](auto q_) AIM_AI {
        constexpr int q = decltype(q_)::value + 1;
        v[q] = tw_mul<false>(v[q], row, q - 1);
      });
      Dft<RM, false, V>::run(v);
      V g[RM];
      spectrum(g, jj);
      static_for<RM>([&](auto p_) AIM_AI {
        constexpr int p = decltype(p_)::value;
        v[p] = cmul(v[p], g[p]);
      });
      Dft<RM, true, V>::run(v);
    };
    if (act) {
      middle(va, beta);
      middle(vb, beta + RM);
    }
    // middle butterfly jj's output p is element p LM + jj (LM = R0); the last
    // stage's butterfly beta reads elements beta R0 + q
    V w[R0];
    static_for<2>([&](auto h_) AIM_AI {
      constexpr int h = decltype(h_)::value;
      constexpr int p0 = h ? S1 : 0, p1 = h ? RM : S1;
      if (act)
        static_for<p1 - p0>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value + p0;
          lds[((p - p0) * LM + beta) * B + b] = va[p];
          lds[((p - p0) * LM + beta + RM) * B + b] = vb[p];
        });
      __syncthreads();
      const V *rowp = lds + ((h ? beta - S1 : beta) * R0) * B + b;
      if (act && (h ? beta >= S1 : beta < S1))
        static_for<R0>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          w[q] = rowp[q * B];
        });
      if constexpr (h == 0) __syncthreads();
    });
    auto st = [&](int i, V x) AIM_AI {
      if (i < n_x) bstore<V, kNtAux>(x, fr, o_beta, t0 + (uint32_t)((i - beta) * es) * SV);
    };
    if (act) stage_compute_store_p<R0, true, false, R0 / 2, true>(w, beta, RM, 1, twr, st);
  } else if constexpr (ML::split) {
    // forward stage 1 (L = 1: no twiddles) -> LDS -> forward stage 2,
    // spectrum, inverse stage 1 in registers -> LDS -> inverse stage 2. Each
    // exchange runs in two halves: butterfly outputs p < S first (read by the
    // next stage's butterflies j < S), then p >= S (butterflies j >= S).
    constexpr int S0 = ML::S0, S1 = ML::S1;
    __syncthreads();  // twiddle tables ready
    if (act0) {
      if constexpr (HALF) dft_upper_zero<R0, false, V>(v0);
      else Dft<R0, false, V>::run(v0);
    }
    V v[RM];
    // stage-1 butterfly beta's output p is element p Mp0 + beta; middle
    // butterfly j reads elements j RM + q (Mp0 = RM)
    auto exchange1 = [&](auto half_) AIM_AI {
      constexpr int h = decltype(half_)::value;
      constexpr int p0 = h ? S0 : 0, p1 = h ? R0 : S0;
      if (act0)
        static_for<p1 - p0>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value + p0;
          lds[((p - p0) * Mp0 + beta) * B + b] = v0[p];
        });
      __syncthreads();
      // (the row's base as its own non-negative index, so the element offsets
      // fold into the LDS instructions)
      const V *rowp = lds + ((h ? j - S0 : j) * RM) * B + b;
      if (act_mid && (h ? j >= S0 : j < S0))
        static_for<RM>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          v[q] = rowp[q * B];
        });
      __syncthreads();
    };
    exchange1(std::integral_constant<int, 0>{});
    exchange1(std::integral_constant<int, 1>{});
    if (act_mid) {
      const V *row = twm + j * (RM - 1);
      static_for<RM - 1>([&](auto q_) AIM_AI {
        constexpr int q = decltype(q_)::value + 1;
        v[q] = tw_mul<false>(v[q], row, q - 1);
      });
      Dft<RM, false, V>::run(v);
      V g[RM];
      spectrum(g, j);
      static_for<RM>([&](auto p_) AIM_AI {
        constexpr int p = decltype(p_)::value;
        v[p] = cmul(v[p], g[p]);
      });
      Dft<RM, true, V>::run(v);
    }
    // middle butterfly j's output p is element p LM + j (LM = R0); the
    // inverse's last stage (radix R0, L = RM, M' = 1) butterfly beta reads
    // elements beta R0 + q
    V w[R0];
    const bool act_last = line_ok && (beta < RM);
    auto exchange2 = [&](auto half_) AIM_AI {
      constexpr int h = decltype(half_)::value;
      constexpr int p0 = h ? S1 : 0, p1 = h ? RM : S1;
      if (act_mid)
        static_for<p1 - p0>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value + p0;
          lds[((p - p0) * LM + j) * B + b] = v[p];
        });
      __syncthreads();
      const V *rowp = lds + ((h ? beta - S1 : beta) * R0) * B + b;
      if (act_last && (h ? beta >= S1 : beta < S1))
        static_for<R0>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          w[q] = rowp[q * B];
        });
      if constexpr (h == 0) __syncthreads();
    };
    exchange2(std::integral_constant<int, 0>{});
    exchange2(std::integral_constant<int, 1>{});
    auto st = [&](int i, V x) AIM_AI {
      if (i < n_x) bstore<V, kNtAux>(x, fr, o_beta, t0 + (uint32_t)((i - beta) * es) * SV);
    };
    if (act_last)
      stage_compute_store_p<R0, true, false, HALF ? R0 / 2 : R0, true>(w, beta, RM, 1, twr, st);
  } else {
    __syncthreads();  // twiddle tables ready
    // first forward stage
    {
      auto st = [&](int i, V x) AIM_AI { lds[i * B + b] = x; };
      if (act0) stage_compute_store_p<R0, false, HALF, R0, false>(v0, beta, 1, Mp0, twl, st);
      __syncthreads();
    }
    // further forward stages but the last (3-stage plans)
    static_for<ns - 2>([&](auto s_) AIM_AI {
      constexpr int s = decltype(s_)::value + 1;
      constexpr int R = PC::r(s), L = PC::lb(s), Mp = P / (L * R), nb = P / R;
      const bool active = line_ok && (beta < nb);
      auto ld = [&](int i) AIM_AI -> V { return lds[i * B + b]; };
      auto st = [&](int i, V x) AIM_AI { lds[i * B + b] = x; };
      V v[R];
      if (active) stage_load<R, false, V>(v, beta, Mp, ld);
      __syncthreads();
      if (active) stage_compute_store<R, false, V>(v, beta, L, Mp, twl, st);
      __syncthreads();
    });
    // last forward stage, spectrum multiply, first inverse stage in registers
    {
      V v[RM];
      if (act_mid)
        static_for<RM>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          v[q] = lds[(j * RM + q) * B + b];
        });
      __syncthreads();
      if (act_mid) {
        if constexpr (ML::rows) {
          const V *row = twm + j * (RM - 1);
          static_for<RM - 1>([&](auto q_) AIM_AI {
            constexpr int q = decltype(q_)::value + 1;
            v[q] = tw_mul<false>(v[q], row, q - 1);
          });
        } else {
          static_for<RM - 1>([&](auto q_) AIM_AI {
            constexpr int q = decltype(q_)::value + 1;
            v[q] = tw_mul<false>(v[q], twl, j * q);
          });
        }
        Dft<RM, false, V>::run(v);
        V g[RM];
        spectrum(g, j);
        static_for<RM>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value;
          v[p] = cmul(v[p], g[p]);
        });
        Dft<RM, true, V>::run(v);
        static_for<RM>([&](auto p_) AIM_AI {
          constexpr int p = decltype(p_)::value;
          lds[(p * LM + j) * B + b] = v[p];
        });
      }
      __syncthreads();
    }
    // remaining inverse stages, radices in reverse order; the last (M' = 1)
    // writes elements beta + L p of its line
    static_for<ns - 1>([&](auto s_) AIM_AI {
      constexpr int s = decltype(s_)::value + 1;
      constexpr int R = PC::ri(s), L = PC::lbi(s), Mp = P / (L * R), nb = P / R;
      constexpr bool last = (s == ns - 1);
      const bool active = line_ok && (beta < nb);
      auto ld = [&](int i) AIM_AI -> V { return lds[i * B + b]; };
      auto st = [&](int i, V x) AIM_AI {
        if constexpr (last) {
          if (i < n_x) bstore<V, kNtAux>(x, fr, o_beta, t0 + (uint32_t)((i - beta) * es) * SV);
        } else {
          lds[i * B + b] = x;
        }
      };
      V v[R];
      if (active) stage_load<R, true, V>(v, beta, Mp, ld);
      if constexpr (!last) __syncthreads();
      if (active)
        stage_compute_store_p<R, true, false, (last && HALF) ? R / 2 : R, last && ML::rows>(
            v, beta, L, Mp, (last && ML::rows) ? twr : twl, st);
      if constexpr (!last) __syncthreads();
    });
  }
}

template <typename T, class PC, bool KYL, int ROW, bool NT>
__global__ void __launch_bounds__((threads_mid<T, PC, ROW, mid_wide_plan<PC>()>()),
                                  (mid_min_waves<T, PC, ROW, mid_wide_plan<PC>()>()))
    k_fft_mid(cx<T> *__restrict__ data, int n_x, int nfield, int Py, int Pz, int ntile, int slots,
              int Hy, int Hz, const cx<T> *__restrict__ ghat, const cx<T> *__restrict__ tw,
              int64_t fstride, FastDiv dfield, FastDiv dtile) {
  mid_body<T, PC, KYL, ROW, mid_wide_plan<PC>(), NT>(data, n_x, nfield, Py, Pz, ntile, slots, Hy,
                                                     Hz, ghat, tw, fstride, dfield, dtile,
                                                     blockIdx.x);
}

// ---------------------------------------------------------------------------
// The y passes and the x pass of a field group in one launch (kz-blocked
// layout, P_x = P_y). The x pass is bound by vector-ALU issue (two FFTs per
// element loaded), the y passes by HBM traffic, so running them side by side
// keeps both busy: the fields are split into G groups and launch t runs the
// x pass of group t - 1 together with the forward y pass of group t and the
// inverse y pass of group t - 2 (G + 2 launches in all). The launch's blocks
// come in runs of 8 (one per XCD); each run has one role, and the roles are
// spread evenly over the launch so every CU mixes them. All roles use the nt
// cache policy (the set-up keeps this launch only where it times faster).
template <typename T>
struct XyStrided {
  const cx<T> *in;
  cx<T> *out;
  int n_in, n_out;
  int64_t inner;
  int ntile;
  LineMap imap, omap;
  int64_t b0, nb;  // first tile of this launch's lines, tiles in it
};
template <typename T>
struct XyMid {
  cx<T> *data;  // first field of the group
  int n_x, nfield, Py, Pz, ntile, slots, Hy, Hz;
  int64_t fstride;
  FastDiv dfield, dtile;
  int64_t nb;  // blocks of the x pass (slots * 8), 0: none in this launch
};

template <typename T, class PC>
constexpr int threads_xy() {
  return threads_mid<T, PC>() > threads_strided<T, PC>() ? threads_mid<T, PC>()
                                                         : threads_strided<T, PC>();
}

template <typename T, class PC, bool PRF, bool PRI>
__global__ void __launch_bounds__((threads_xy<T, PC>()), (sizeof(T) == 4 ? 4 : 3))
    k_fft_xy(XyMid<T> xm, XyStrided<T> yf, XyStrided<T> yi, const cx<T> *__restrict__ ghat,
             const cx<T> *__restrict__ twx, const cx<T> *__restrict__ twy, int64_t nruns,
             int64_t yruns) {
  const int64_t run = blockIdx.x / kXcd, xcd = blockIdx.x % kXcd;
  const int64_t ylo = run * yruns / nruns, yhi = (run + 1) * yruns / nruns;
  if (yhi > ylo) {  // a y run: forward tiles first, then inverse ones
    const int64_t v = ylo * kXcd + xcd;
    if (v < yf.nb)
      strided_body<T, false, PRF, PC>(yf.in, yf.out, yf.n_in, yf.n_out, yf.inner, yf.ntile,
                                      yf.imap, yf.omap, twy, yf.b0 + v);
    else if (v - yf.nb < yi.nb)
      strided_body<T, true, PRI, PC>(yi.in, yi.out, yi.n_in, yi.n_out, yi.inner, yi.ntile,
                                     yi.imap, yi.omap, twy, yi.b0 + (v - yf.nb));
    return;
  }
  const int64_t v = (run - ylo) * kXcd + xcd;  // x runs keep the XCD of their block
  if (v < xm.nb)
    mid_body<T, PC, false>(xm.data, xm.n_x, xm.nfield, xm.Py, xm.Pz, xm.ntile, xm.slots, xm.Hy,
                           xm.Hz, ghat, twx, xm.fstride, xm.dfield, xm.dtile, v);
}

template <typename T, class PC>
void launch_contig(const cx<T> *in, cx<T> *out, int n_in, int n_out, int64_t lines,
                   const ContigMap &imap, const ContigMap &omap, bool inverse, const cx<T> *tw,
                   hipStream_t s) {
  constexpr int B = tile_contig<T, PC>();
  constexpr int threads = threads_contig<T, PC>();
  const size_t lds = PC::ns > 1 ? ((size_t)B * (PC::P + 1) + PC::P) * sizeof(cx<T>) : 0;
  const int64_t blocks = (lines + B - 1) / B;
  // a tile narrower than the fields of a line: ranges per XCD (measured on the
  // in-plane inverse y pass, whose field-interleaved stores otherwise leave
  // partly written lines in four L2s: 128-lambda plate 71 -> 54 us); wider
  // tiles keep the plain numbering
  const int64_t slots =
      (B < std::max(imap.fin, omap.fin)) ? (blocks + kXcd - 1) / kXcd : 0;
  const int64_t launched = slots ? slots * kXcd : blocks;
  if (launched > INT32_MAX) throw Error(AIM_ERR_ARG, "contiguous pass: too many lines");
  // 32-bit line arithmetic and element offsets in the kernel
  if (contig_line_bound(imap, lines) >= INT32_MAX || contig_line_bound(omap, lines) >= INT32_MAX ||
      (int64_t)PC::P * std::max(imap.es, omap.es) >= INT32_MAX)
    throw Error(AIM_ERR_ARG, "contiguous pass: lines or line lengths beyond 32-bit offsets");
  const bool pr = pass_prunable<PC>(inverse, n_in, n_out);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)launched), dim3(threads), lds, s, in, out, n_in,
                       n_out, lines, imap, omap, tw, B, slots);
  };
  if (inverse)
    pr ? go(k_fft_contig<T, true, true, PC>) : go(k_fft_contig<T, true, false, PC>);
  else
    pr ? go(k_fft_contig<T, false, true, PC>) : go(k_fft_contig<T, false, false, PC>);
  LAUNCHCHECK();
}

template <typename T, class PC, int ROW>
void launch_strided_rows(const cx<T> *in, cx<T> *out, int n_in, int n_out, int64_t outer,
                         int64_t inner, const LineMap &imap, const LineMap &omap, bool inverse,
                         const cx<T> *tw, hipStream_t s) {
  constexpr int B = tile_strided<T, PC, ROW>();
  constexpr int threads = threads_strided<T, PC, ROW>();
  const int ntile = (int)((inner + B - 1) / B);
  const size_t lds = PC::ns > 1 ? (size_t)PC::P * (B + 1) * sizeof(cx<T>) : 0;
  const int64_t blocks = outer * ntile;
  const int64_t slots = ROW < 128 ? (blocks + kXcd - 1) / kXcd : 0;
  const int64_t launched = ROW < 128 ? slots * kXcd : blocks;
  if (launched > INT32_MAX || inner >= INT32_MAX)
    throw Error(AIM_ERR_ARG, "strided pass: too many tiles or lines");
  const bool pr = pass_prunable<PC>(inverse, n_in, n_out);
  // 64-byte tiles keep the default policy: the two tiles of a 128-byte line
  // meet in L2, which the nt policy would evict between them
  const bool nt =
      ROW == 128 &&
      (uint64_t)outer * (uint64_t)inner * (uint64_t)std::max(n_in, n_out) * sizeof(cx<T>) >
          kStreamBytes;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)launched), dim3(threads), lds, s, in, out, n_in,
                       n_out, inner, ntile, imap, omap, tw, blocks, slots);
  };
  auto pick = [&](auto nt_) {
    constexpr bool NT = decltype(nt_)::value;
    if (inverse)
      pr ? go(k_fft_strided<T, true, true, PC, ROW, NT>)
         : go(k_fft_strided<T, true, false, PC, ROW, NT>);
    else
      pr ? go(k_fft_strided<T, false, true, PC, ROW, NT>)
         : go(k_fft_strided<T, false, false, PC, ROW, NT>);
  };
  if constexpr (ROW == 128)
    nt ? pick(std::true_type{}) : pick(std::false_type{});
  else
    pick(std::false_type{});
  LAUNCHCHECK();
}

// row_bytes: 128 or 64 (the tile of consecutive lines per work-group)
template <typename T, class PC>
void launch_strided(const cx<T> *in, cx<T> *out, int n_in, int n_out, int64_t outer, int64_t inner,
                    const LineMap &imap, const LineMap &omap, bool inverse, const cx<T> *tw,
                    int row_bytes, hipStream_t s) {
  if (row_bytes == 64)
    launch_strided_rows<T, PC, 64>(in, out, n_in, n_out, outer, inner, imap, omap, inverse, tw, s);
  else
    launch_strided_rows<T, PC, 128>(in, out, n_in, n_out, outer, inner, imap, omap, inverse, tw, s);
}

template <typename T, class PC, int ROW>
void launch_mid_rows(cx<T> *data, int n_x, int nfield, int Py, int Pz, int Hy, int Hz,
                     const cx<T> *ghat, const cx<T> *tw, int blk, int64_t fstride, hipStream_t s) {
  constexpr bool WIDE = mid_wide_plan<PC>();
  constexpr int B = MidLds<T, PC, ROW, WIDE>::B;  // lines per work-group
  constexpr int threads = threads_mid<T, PC, ROW, WIDE>();
  const bool kyl = blk == 0;
  if (PC::r(0) % 2 == 0 && 2 * n_x > PC::P)  // the half-pruned first/last stages need it
    throw Error(AIM_ERR_ARG, "x pass: more than P/2 sources on a line");
  if (blk < 0 || (!kyl && blk != kGridBlock<T>) ||
      (!kyl && (B <= blk ? blk % B : B % blk) != 0))
    throw Error(AIM_ERR_ARG, "x pass: kz block other than 128 bytes, or not tiled by the lines");
  // 32-bit buffer offsets: the kz blocks of a work-group (a kz plane) of a
  // field, and the octant
  const uint64_t wblocks = (!kyl && B > blk) ? (uint64_t)(B / blk) : 1;
  if ((uint64_t)n_x * Py * (kyl ? 1 : blk) * wblocks * sizeof(cx<T>) >= (1ull << 31) ||
      (uint64_t)Hy * Hz * (PC::P / 2 + 1) * sizeof(cx<T>) >= (1ull << 31))
    throw Error(AIM_ERR_ARG, "x pass: grid too large for 32-bit offsets");
  const int Pt = kyl ? Py : Pz, Pf = kyl ? Pz : Py;  // tile axis, fixed axis
  const int ntile = (Pt + B - 1) / B;
  const size_t lds = (size_t)MidLds<T, PC, ROW, WIDE>::total * sizeof(cx<T>);
  // work items (folded fixed index 0 .. Pf/2, tile, mirror, field), dealt to
  // the XCDs in 8 contiguous ranges
  const int64_t items = 2 * ((int64_t)Pf / 2 + 1) * ntile * nfield;
  const int64_t slots = (items + kXcd - 1) / kXcd;
  if (slots * kXcd > INT32_MAX) throw Error(AIM_ERR_ARG, "x pass: too many tiles");
  // the nt policy as in the y passes: 128-byte tiles of grids beyond the
  // last-level cache
  const uint64_t grid_bytes = (uint64_t)nfield * Py * Pz * n_x * sizeof(cx<T>);
  const FastDiv dfield = make_fastdiv((uint32_t)nfield), dtile = make_fastdiv((uint32_t)ntile);
  const bool nt = ROW == 128 && grid_bytes > kStreamBytes;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)(slots * kXcd)), dim3(threads), lds, s, data, n_x,
                       nfield, Py, Pz, ntile, (int)slots, Hy, Hz, ghat, tw, fstride, dfield, dtile);
  };
  if (kyl)
    go(k_fft_mid<T, PC, true, ROW, false>);
  else if constexpr (ROW == 128)
    nt ? go(k_fft_mid<T, PC, false, ROW, true>) : go(k_fft_mid<T, PC, false, ROW, false>);
  else
    go(k_fft_mid<T, PC, false, ROW, false>);
  LAUNCHCHECK();
}

// blk > 0: kz-blocked layout [nfield][ceil(Pz/blk)][n_x][Py][blk], tiles of
// consecutive kz; blk == 0: thin layout [nfield][Pz][n_x][Py] (few kz, as
// for a flat scatterer), tiles of consecutive ky. row_bytes: 128 or 64.
template <typename T, class PC>
void launch_mid(cx<T> *data, int n_x, int nfield, int Py, int Pz, int Hy, int Hz,
                const cx<T> *ghat, const cx<T> *tw, int blk, int64_t fstride, int row_bytes,
                hipStream_t s) {
  if (row_bytes == 64)
    launch_mid_rows<T, PC, 64>(data, n_x, nfield, Py, Pz, Hy, Hz, ghat, tw, blk, fstride, s);
  else
    launch_mid_rows<T, PC, 128>(data, n_x, nfield, Py, Pz, Hy, Hz, ghat, tw, blk, fstride, s);
}

// The pipelined y, x and y passes of the kz-blocked layout (see k_fft_xy):
// forward y pass gz -> g2 (line maps m1y -> m2), x pass with the spectrum on
// g2 in place, inverse y pass g2 -> g1 (m2 -> m1y), over F fields in G groups.
template <typename T, class PC>
void launch_xy(const cx<T> *gz, cx<T> *g2, cx<T> *g1, int Nx, int Ny, int F, int G, int Py,
               int Pz, int Hy, int Hz, const cx<T> *ghat, const cx<T> *twx, const cx<T> *twy,
               int blk, int64_t V2, const LineMap &m1y, const LineMap &m2, hipStream_t s) {
  constexpr int B = tile_mid<T, PC>();
  static_assert(tile_strided<T, PC>() == B, "x and y tiles differ");
  constexpr int threads = threads_xy<T, PC>();
  constexpr bool PRF = PC::r(0) % 2 == 0, PRI = PC::r(PC::ns - 1) % 2 == 0;
  if (G < 1 || F % G != 0) throw Error(AIM_ERR_ARG, "y/x pipeline: groups do not divide the fields");
  if (Py != PC::P) throw Error(AIM_ERR_ARG, "y/x pipeline: x and y lengths differ");
  // pruned first / last stages: at most P/2 sources per x and y line
  if ((PRF || PRI) && (2 * Nx > PC::P || 2 * Ny > PC::P))
    throw Error(AIM_ERR_ARG, "y/x pipeline: more than P/2 sources on a line");
  if (blk != kGridBlock<T> || blk % B != 0)
    throw Error(AIM_ERR_ARG, "y/x pipeline: kz block other than 128 bytes, or not tiled");
  if ((uint64_t)Nx * Py * blk * sizeof(cx<T>) >= (1ull << 31) ||
      (uint64_t)Hy * Hz * (PC::P / 2 + 1) * sizeof(cx<T>) >= (1ull << 31))
    throw Error(AIM_ERR_ARG, "y/x pipeline: grid too large for 32-bit offsets");
  const int Fg = F / G;
  const int ntile = (Pz + B - 1) / B;  // kz tiles (both passes)
  const int64_t ynb = (int64_t)Fg * Nx * ntile;
  const int64_t items = 2 * ((int64_t)Py / 2 + 1) * ntile * Fg;
  const int64_t slots = (items + kXcd - 1) / kXcd;
  if (slots * kXcd > INT32_MAX) throw Error(AIM_ERR_ARG, "y/x pipeline: too many tiles");
  const size_t lds = (size_t)std::max(MidLds<T, PC>::total, PC::P * (B + 1)) * sizeof(cx<T>);
  for (int t = 0; t <= G + 1; ++t) {
    XyMid<T> xm{};
    if (t >= 1 && t <= G) {
      xm.data = g2 + (int64_t)(t - 1) * Fg * V2;
      xm.n_x = Nx;
      xm.nfield = Fg;
      xm.Py = Py;
      xm.Pz = Pz;
      xm.ntile = ntile;
      xm.slots = (int)slots;
      xm.Hy = Hy;
      xm.Hz = Hz;
      xm.fstride = V2;
      xm.dfield = make_fastdiv((uint32_t)Fg);
      xm.dtile = make_fastdiv((uint32_t)ntile);
      xm.nb = slots * kXcd;
    }
    XyStrided<T> yf{gz, g2, Ny, Py, Pz, ntile, m1y, m2, (int64_t)t * ynb, t < G ? ynb : 0};
    XyStrided<T> yi{g2, g1, Py, Ny, Pz, ntile, m2, m1y, (int64_t)(t - 2) * ynb,
                    (t >= 2 && t - 2 < G) ? ynb : 0};
    const int64_t xruns = xm.nb / kXcd;
    const int64_t yruns = (yf.nb + yi.nb + kXcd - 1) / kXcd;
    const int64_t nruns = xruns + yruns;
    if (nruns == 0) continue;
    if (nruns * kXcd > INT32_MAX) throw Error(AIM_ERR_ARG, "y/x pipeline: launch too large");
    hipLaunchKernelGGL((k_fft_xy<T, PC, PRF, PRI>), dim3((unsigned)(nruns * kXcd)), dim3(threads),
                       lds, s, xm, yf, yi, ghat, twx, twy, nruns, yruns);
    LAUNCHCHECK();
  }
}

[[noreturn]] inline void bad_length(int P) {
  throw Error(AIM_ERR_ARG, "no FFT kernels for length " + std::to_string(P));
}

}  // namespace fftk

}  // namespace aim
