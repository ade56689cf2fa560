// Line addressing of the strided FFT passes (shared by the passes and their
// callers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace aim {
namespace fftk {

// Address of element i of line (o, c) of a strided pass, with o the outer
// line index and c the contiguous line index. With o = o_hi * lo_count + o_lo:
//   plain   (blk == 0): o_hi*hi + o_lo*lo + c            + i*elem
//   blocked (blk  > 0): o_hi*hi + o_lo*lo + (c/blk)*bstr + c%blk + i*blk
// The blocked form stores the contiguous index in runs of blk (128 bytes), so
// the lines of one work-group lie close together in memory.
struct LineMap {
  int64_t hi, lo, bstr, elem;
  int lo_count, blk;
  // optional element range per line: a line with outer index o holds
  // elements range[2 r] <= i < range[2 r + 1] only, r = o % range_rows (the
  // others read as zero on input and are not stored on output)
  const int32_t *range = nullptr;
  int range_rows = 0;
};
inline LineMap with_range(LineMap m, const int32_t *range, int rows) {
  m.range = range;
  m.range_rows = rows;
  return m;
}
// Division of numerators below 2^31 by a run-time divisor d >= 1 as a
// multiply-high, an add and a shift (the round-up method of Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994):
// with s = ceil(log2 d) and m = floor(2^32 (2^s - d) / d) + 1,
// n / d = (mulhi(n, m) + n) >> s. A work-group-uniform numerator then divides
// in scalar instructions instead of the vector ALU's reciprocal sequence.
struct FastDiv {
  uint32_t d = 1, m = 0, s = 0;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  while ((1ull << f.s) < d) ++f.s;
  f.m = (uint32_t)((((1ull << f.s) - d) << 32) / d + 1);
  return f;
}
__host__ __device__ inline uint32_t fast_div(uint32_t n, const FastDiv &f) {
  const uint32_t h = (uint32_t)(((uint64_t)n * f.m) >> 32);
  return (h + n) >> f.s;
}

// (outer and inner line indices stay below 2^31, checked by the launcher:
// the index arithmetic divides in 32 bits, only the offsets are 64-bit)
__host__ __device__ inline int64_t line_base(const LineMap &m, int64_t o, int64_t c) {
  const uint32_t ou = (uint32_t)o, lc = (uint32_t)m.lo_count, oh = ou / lc, ol = ou - oh * lc;
  const int64_t b = (int64_t)oh * m.hi + (int64_t)ol * m.lo;
  if (m.blk == 0) return b + c;
  const uint32_t cu = (uint32_t)c, bk = (uint32_t)m.blk, cb = cu / bk;
  return b + (int64_t)cb * m.bstr + (int64_t)(cu - cb * bk);
}
__host__ __device__ inline int64_t line_elem(const LineMap &m) { return m.blk == 0 ? m.elem : m.blk; }

// plain line map: line (o, c) starts at o * outer + c, elements elem apart
inline LineMap plain_map(int64_t outer, int64_t elem) {
  LineMap m{};
  m.hi = outer;
  m.lo = 0;
  m.bstr = 0;
  m.elem = elem;
  m.lo_count = 1;
  m.blk = 0;
  return m;
}

// kz-blocked grid [F][ceil(Pz/blk)][Nx][Py][blk] seen by the y passes: outer
// o = f * Nx + x, contiguous index kz, element ky
inline LineMap blocked_map(int64_t field_stride, int Nx, int Py, int blk) {
  LineMap m{};
  m.hi = field_stride;
  m.lo = (int64_t)Py * blk;
  m.bstr = (int64_t)Nx * Py * blk;
  m.elem = 0;
  m.lo_count = Nx;
  m.blk = blk;
  return m;
}

// Line addressing of the contiguous passes: line L = f per + l starts at
// f fs + l ls (per = 0: no split, L ls), its elements es apart.
// With sel, a pass runs only the selected lines of each field: pass line L is
// line (L / nsel) sper + sel[L % nsel] of the full numbering (sper lines per
// field), which the map then addresses (device side only).
struct ContigMap {
  int64_t per, fs, ls, es;
  const int32_t *sel = nullptr;
  int64_t nsel = 0, sper = 0;
  // optional element ranges of each selected line s: elements
  // range[4 s] <= i < range[4 s + 1] and range[4 s + 2] <= i < range[4 s + 3]
  // only (the others read as zero on input, are not stored on output)
  const int32_t *range = nullptr;
  // fin > 0: fields innermost in the pass numbering, L = l fin + f (the
  // fields of one line are consecutive pass lines): line l (through sel if
  // given, sel index l) of field f starts at f fs + l ls; per is unused
  int64_t fin = 0;
};
// Pass lines, and lines of the full numbering, stay below 2^31 (the launcher
// checks it), so the line arithmetic divides in 32 bits; only the element
// offsets are 64-bit.
// index into sel / range of pass line L
__host__ __device__ inline int64_t sel_index(const ContigMap &m, int64_t L) {
  const uint32_t Lu = (uint32_t)L;
  return m.fin ? (int64_t)(Lu / (uint32_t)m.fin) : (int64_t)(Lu % (uint32_t)m.nsel);
}
__host__ __device__ inline int64_t contig_base(const ContigMap &m, int64_t L) {
  const uint32_t Lu = (uint32_t)L;
  if (m.fin) {
    const uint32_t fin = (uint32_t)m.fin, l = Lu / fin, f = Lu - l * fin;
    return (int64_t)f * m.fs + (m.sel ? (int64_t)m.sel[l] : (int64_t)l) * m.ls;
  }
  uint32_t line = Lu;
  if (m.sel) {
    const uint32_t ns = (uint32_t)m.nsel, f = Lu / ns;
    line = f * (uint32_t)m.sper + (uint32_t)m.sel[Lu - f * ns];
  }
  if (m.per == 0) return (int64_t)line * m.ls;
  const uint32_t per = (uint32_t)m.per, f = line / per;
  return (int64_t)f * m.fs + (int64_t)(line - f * per) * m.ls;
}
// the largest line index of the full numbering that pass lines 0 .. lines - 1
// reach through m (host side, for the launcher's 32-bit check)
inline int64_t contig_line_bound(const ContigMap &m, int64_t lines) {
  if (m.fin) return lines;
  if (m.sel) return (lines / m.nsel + 1) * m.sper;
  return lines;
}
// lines ls apart, elements adjacent
inline ContigMap contig_map(int64_t ls) { return ContigMap{0, 0, ls, 1}; }
// per lines of each of the fields fs apart, lines ls apart, elements es apart
inline ContigMap contig_map(int64_t per, int64_t fs, int64_t ls, int64_t es) {
  return ContigMap{per, fs, ls, es};
}
// fields innermost: line l of field f at f fs + l ls (pass line l fin + f),
// elements es apart, optionally over the selected lines sel[0 .. nsel) and
// their element ranges
inline ContigMap fields_inner(int64_t fin, int64_t fs, int64_t ls, int64_t es,
                              const int32_t *sel = nullptr, int64_t nsel = 0,
                              const int32_t *range = nullptr) {
  ContigMap m{0, fs, ls, es};
  m.fin = fin;
  m.sel = sel;
  m.nsel = nsel;
  m.range = range;
  return m;
}
// the same map over the selected lines sel[0 .. nsel) of each field of sper lines
inline ContigMap select_lines(ContigMap m, const int32_t *sel, int64_t nsel, int64_t sper,
                              const int32_t *range = nullptr) {
  m.sel = sel;
  m.nsel = nsel;
  m.sper = sper;
  m.range = range;
  return m;
}

}  // namespace fftk
}  // namespace aim
