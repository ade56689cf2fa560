// Host phase of plan construction: mesh validation, RWG table, AIM grid,
// stencil anchors, near-zone CSR pattern and FFT length selection.
//
// This translation unit is plain C++ (no GPU calls) so that it can run on
// machines without a GPU. It is compiled with -ffp-contract=off: the integer
// decisions it takes from floating point (anchor rounding, the near-zone
// distance test) must not depend on fused multiply-adds.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <thread>

#include "aim_internal.h"
#include "fft_plans.h"

namespace aim {

// ---------------------------------------------------------------------------
// FFT lengths: the table of lengths with compiled kernel sets.
bool fft_plan_for(int P, FftPlan *out) {
  switch (P) {
#define AIM_X(L, a, b, c)                                 \
  case L: {                                               \
    FftPlan pl;                                           \
    pl.P = L;                                             \
    pl.ns = (b == 1) ? 1 : ((c == 1) ? 2 : 3);            \
    pl.r[0] = a;                                          \
    pl.r[1] = b;                                          \
    pl.r[2] = c;                                          \
    *out = pl;                                            \
    return true;                                          \
  }
    AIM_FOR_EACH_FFT_PLAN(AIM_X)
#undef AIM_X
    default:
      return false;
  }
}

int fft_length_at_least(int lo) {
  static const int lengths[] = {
#define AIM_X(L, a, b, c) L,
      AIM_FOR_EACH_FFT_PLAN(AIM_X)
#undef AIM_X
  };
  for (int L : lengths)
    if (L >= lo) return L;
  return -1;
}

// ---------------------------------------------------------------------------
static void fail_mesh(const std::string &m) { throw Error(AIM_ERR_MESH, m); }
static void fail_arg(const std::string &m) { throw Error(AIM_ERR_ARG, m); }

void host_plan_build(const aim_mesh &m, const aim_params &p, HostPlan *hp) {
  if (!(m.freq_hz > 0)) fail_arg("freq_hz must be > 0");
  if (m.nv <= 0 || m.nt <= 0 || !m.verts || !m.tris) fail_arg("empty mesh");
  if (!(p.h_lambda > 0)) fail_arg("h_lambda must be > 0");
  if (p.order < 1 || p.order > 5) fail_arg("order must be in 1..5");
  if (p.quad_points != 0 && p.quad_points != 7) fail_arg("quad_points must be 7 (or 0)");
  if (!(p.near_radius_lambda >= 0)) fail_arg("near_radius_lambda must be >= 0");
  const bool cfie_all = (p.flags & AIM_FLAG_CFIE) != 0;
  const bool cfie_closed = (p.flags & AIM_FLAG_CFIE_CLOSED) != 0;
  if ((cfie_all || cfie_closed) && !(p.cfie_alpha >= 0.0 && p.cfie_alpha <= 1.0))
    fail_arg("cfie_alpha must be in [0, 1]");
  if (m.nv > INT32_MAX || m.nt > INT32_MAX) fail_arg("mesh too large");

  HostPlan &h = *hp;
  h.nv = m.nv;
  h.nt = m.nt;
  h.freq = m.freq_hz;
  h.lam = kC0 / m.freq_hz;
  h.k = 2.0 * kPi * m.freq_hz / kC0;
  h.h = p.h_lambda * h.lam;
  h.r_near = p.near_radius_lambda * h.lam;
  h.order = p.order;
  h.K = (p.order + 1) * (p.order + 1) * (p.order + 1);
  h.verts.assign(m.verts, m.verts + 3 * m.nv);
  h.tris.assign(m.tris, m.tris + 3 * m.nt);
  for (double v : h.verts)
    if (!std::isfinite(v)) fail_mesh("non-finite vertex coordinate");

  // triangles: index range, distinct vertices, area
  const int64_t nt = m.nt;
  h.area.resize(nt);
  const double min_area = 1e-12 * h.lam * h.lam;
  for (int64_t t = 0; t < nt; ++t) {
    int a = h.tris[3 * t], b = h.tris[3 * t + 1], c = h.tris[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= m.nv || b >= m.nv || c >= m.nv)
      fail_mesh("vertex index out of range in triangle " + std::to_string(t));
    if (a == b || b == c || a == c) fail_mesh("triangle with repeated vertex " + std::to_string(t));
    const double *A = &h.verts[3 * a], *B = &h.verts[3 * b], *C = &h.verts[3 * c];
    double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    h.area[t] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(h.area[t] > min_area)) fail_mesh("degenerate triangle " + std::to_string(t));
  }

  // edges: (lo, hi, triangle, local vertex opposite the edge, 1 if the
  // triangle runs the edge from lo to hi), sorted
  struct E {
    int32_t lo, hi, t, i, fwd;
  };
  std::vector<E> e(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) {
      int a = h.tris[3 * t + (i + 1) % 3], b = h.tris[3 * t + (i + 2) % 3];
      e[3 * t + i] = {std::min(a, b), std::max(a, b), (int32_t)t, i, a < b ? 1 : 0};
    }
  std::sort(e.begin(), e.end(), [](const E &x, const E &y) {
    if (x.lo != y.lo) return x.lo < y.lo;
    if (x.hi != y.hi) return x.hi < y.hi;
    return x.t < y.t;
  });
  bool closed = true;  // every edge shared by two triangles that run it in opposite directions
  for (size_t s = 0; s < e.size();) {
    size_t q = s + 1;
    while (q < e.size() && e[q].lo == e[s].lo && e[q].hi == e[s].hi) ++q;
    if (q - s > 2) fail_mesh("edge shared by more than two triangles");
    if (q - s != 2 || e[s].fwd == e[s + 1].fwd) closed = false;
    if (q - s == 2) {
      h.e_lo.push_back(e[s].lo);
      h.e_hi.push_back(e[s].hi);
      h.tp.push_back(e[s].t);
      h.tm.push_back(e[s + 1].t);
      h.vp.push_back(h.tris[3 * (int64_t)e[s].t + e[s].i]);
      h.vm.push_back(h.tris[3 * (int64_t)e[s + 1].t + e[s + 1].i]);
    }
    s = q;
  }
  const int64_t n = (int64_t)h.e_lo.size();
  if (n == 0) fail_mesh("mesh has no interior edge");
  if (cfie_all || cfie_closed) {
    // enclosed volume sum v0 . (v1 x v2) / 6 > 0 for outward normals
    double vol = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
      const double *A = &h.verts[3 * (int64_t)h.tris[3 * t]], *B = &h.verts[3 * (int64_t)h.tris[3 * t + 1]],
                   *C = &h.verts[3 * (int64_t)h.tris[3 * t + 2]];
      vol += A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
             A[2] * (B[0] * C[1] - B[1] * C[0]);
    }
    const bool outward = closed && vol > 0.0;
    if (cfie_all && !outward)
      fail_mesh("the combined-field equation needs a closed, consistently oriented mesh with "
                "outward normals");
    h.cfie = outward;
    h.alpha = outward ? p.cfie_alpha : 1.0;
  }
  h.n = n;
  h.len.resize(n);
  h.centre.resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double *A = &h.verts[3 * (int64_t)h.e_lo[i]], *B = &h.verts[3 * (int64_t)h.e_hi[i]];
    double d0 = A[0] - B[0], d1 = A[1] - B[1], d2 = A[2] - B[2];
    h.len[i] = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    for (int c = 0; c < 3; ++c) {
      // centroids as ((v0 + v1) + v2) / 3, centre as their mean
      const int32_t *tp = &h.tris[3 * (int64_t)h.tp[i]], *tm = &h.tris[3 * (int64_t)h.tm[i]];
      double cp = (h.verts[3 * (int64_t)tp[0] + c] + h.verts[3 * (int64_t)tp[1] + c] +
                   h.verts[3 * (int64_t)tp[2] + c]) / 3.0;
      double cm = (h.verts[3 * (int64_t)tm[0] + c] + h.verts[3 * (int64_t)tm[1] + c] +
                   h.verts[3 * (int64_t)tm[2] + c]) / 3.0;
      h.centre[3 * i + c] = 0.5 * (cp + cm);
    }
  }

  // grid: N_d = max(ceil(extent/h - 1e-9) + 1, M + 1), centred on the box
  const int M = p.order;
  for (int c = 0; c < 3; ++c) {
    double lo = h.verts[c], hi = h.verts[c];
    for (int64_t v = 0; v < m.nv; ++v) {
      lo = std::min(lo, h.verts[3 * v + c]);
      hi = std::max(hi, h.verts[3 * v + c]);
    }
    double ext = hi - lo;
    int64_t nd = std::max<int64_t>((int64_t)std::ceil(ext / h.h - 1e-9) + 1, M + 1);
    if (nd > (1 << 20)) fail_arg("grid too large");
    h.grid[c] = (int)nd;
    double ctr = 0.5 * (hi + lo);
    h.x0[c] = ctr - 0.5 * (double)(nd - 1) * h.h;
    int lo_pad = 2 * (int)nd - 1;
    if (p.fft_min_pad > lo_pad) lo_pad = p.fft_min_pad;
    h.pad[c] = fft_length_at_least(lo_pad);
    if (h.pad[c] < 0) fail_arg("grid dimension beyond the largest supported FFT length");
  }
  int64_t V0 = (int64_t)h.grid[0] * h.grid[1] * h.grid[2];
  int64_t Vp = (int64_t)h.grid[0] * h.pad[1] * h.pad[2];
  const int64_t Vf = (int64_t)h.pad[0] * h.pad[1] * h.pad[2];  // Green's spectrum set-up grid
  if (V0 > INT32_MAX / 2 || Vp > INT32_MAX / 2 || Vf > INT32_MAX / 2)
    fail_arg("grid too large for 32-bit indexing");

  // anchors: round-half-up((c - x0)/h) - M/2 (even M), floor(.) - (M-1)/2 (odd M), clamped
  h.anchor.resize(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      double t = (h.centre[3 * i + c] - h.x0[c]) / h.h;
      int64_t a = (M % 2 == 0) ? (int64_t)std::floor(t + 0.5) - M / 2
                               : (int64_t)std::floor(t) - (M - 1) / 2;
      a = std::min<int64_t>(std::max<int64_t>(a, 0), h.grid[c] - M - 1);
      h.anchor[3 * i + c] = (int32_t)a;
    }

  // near zone: |c_m - c_n|^2 <= r^2 with a uniform cell hash
  const double r = h.r_near, r2 = r * r;
  double bmin[3], bmax[3];
  for (int c = 0; c < 3; ++c) {
    bmin[c] = bmax[c] = h.centre[c];
    for (int64_t i = 0; i < n; ++i) {
      bmin[c] = std::min(bmin[c], h.centre[3 * i + c]);
      bmax[c] = std::max(bmax[c], h.centre[3 * i + c]);
    }
  }
  double span = std::max({bmax[0] - bmin[0], bmax[1] - bmin[1], bmax[2] - bmin[2], 1e-30});
  double cs = std::max(r, span / 256.0);
  int nc[3];
  for (int c = 0; c < 3; ++c) nc[c] = std::max(1, (int)std::floor((bmax[c] - bmin[c]) / cs) + 1);
  const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  std::vector<int32_t> cell_of(n);
  std::vector<int64_t> cstart(ncell + 1, 0);
  auto cidx = [&](int64_t i, int c) {
    int v = (int)std::floor((h.centre[3 * i + c] - bmin[c]) / cs);
    return std::min(std::max(v, 0), nc[c] - 1);
  };
  for (int64_t i = 0; i < n; ++i) {
    cell_of[i] = (int32_t)(((int64_t)cidx(i, 0) * nc[1] + cidx(i, 1)) * nc[2] + cidx(i, 2));
    cstart[cell_of[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  std::vector<int32_t> members(n);
  {
    std::vector<int64_t> fill(cstart.begin(), cstart.end() - 1);
    for (int64_t i = 0; i < n; ++i) members[fill[cell_of[i]]++] = (int32_t)i;
  }
  const int reach = (int)std::ceil(r / cs);
  unsigned nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::vector<int32_t>> part_cols(nthr);
  std::vector<int64_t> count(n, 0);
  auto worker = [&](unsigned tid) {
    int64_t lo = n * tid / nthr, hi = n * (tid + 1) / nthr;
    std::vector<int32_t> &out = part_cols[tid];
    std::vector<int32_t> row;
    for (int64_t i = lo; i < hi; ++i) {
      row.clear();
      int ci[3] = {cidx(i, 0), cidx(i, 1), cidx(i, 2)};
      const double *ca = &h.centre[3 * i];
      for (int a = std::max(0, ci[0] - reach); a <= std::min(nc[0] - 1, ci[0] + reach); ++a)
        for (int b = std::max(0, ci[1] - reach); b <= std::min(nc[1] - 1, ci[1] + reach); ++b)
          for (int d = std::max(0, ci[2] - reach); d <= std::min(nc[2] - 1, ci[2] + reach); ++d) {
            int64_t cell = ((int64_t)a * nc[1] + b) * nc[2] + d;
            for (int64_t s = cstart[cell]; s < cstart[cell + 1]; ++s) {
              int32_t j = members[s];
              const double *cb = &h.centre[3 * (int64_t)j];
              double d0 = ca[0] - cb[0], d1 = ca[1] - cb[1], d2 = ca[2] - cb[2];
              double dd = d0 * d0 + d1 * d1 + d2 * d2;
              if (dd <= r2 || j == i) row.push_back(j);
            }
          }
      std::sort(row.begin(), row.end());
      count[i] = (int64_t)row.size();
      out.insert(out.end(), row.begin(), row.end());
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nthr; ++t) th.emplace_back(worker, t);
  for (auto &t : th) t.join();
  h.rowptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) h.rowptr[i + 1] = h.rowptr[i] + count[i];
  h.nnz = h.rowptr[n];
  if (h.nnz > INT32_MAX) fail_arg("near zone too large for 32-bit indexing");
  h.cols.resize(h.nnz);
  int64_t pos = 0;
  for (unsigned t = 0; t < nthr; ++t) {
    std::memcpy(&h.cols[pos], part_cols[t].data(), part_cols[t].size() * sizeof(int32_t));
    pos += (int64_t)part_cols[t].size();
  }
}

}  // namespace aim
