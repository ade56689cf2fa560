// Restarted GMRES with right Jacobi preconditioning (the matvec's caller).
//
// The paper solves with a diagonal preconditioner and stops on the relative
// RMS residual (Section 2.2). Here every (mesh, plane wave) pair is its own
// system; all systems advance in lock-step so one batched AIM product serves
// them all. Arnoldi runs in FP64 on the device (classical Gram-Schmidt, two
// passes), and so do the Givens rotations and the residual estimate; the host
// only polls the per-system active flags every few iterations. The steps
// between two polls are captured once into a HIP graph and replayed (the
// launch sequence of a segment depends only on its step range, the precision
// and the buffers, which persist in the plan across solves). For AIM_MIXED the
// inner solves use the c64 operator on c128 Krylov vectors, inside an FP64
// iterative-refinement loop r = b - A64 x that decides convergence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <map>
#include <tuple>

#include "aim_internal.h"

namespace aim {

namespace {

constexpr int kRed = 256;

__device__ inline double2 block_sum2(double a, double b) {
  __shared__ double sa[kRed / 64], sb[kRed / 64];
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  double ra = 0, rb = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      ra += sa[i];
      rb += sb[i];
    }
  return make_double2(ra, rb);
}

// All nv dot products of one Gram-Schmidt pass in one launch: every thread
// keeps its kRows entries of w in registers and walks a group of kGroup basis
// vectors (blockIdx.z); each wave writes its partial sum of conj(V[i][r][row])
// w[r][row] to part[(i S + s) np_stride + p], p = the wave's index, and
// k_part_reduce adds the partials in a fixed order: no atomics, bitwise
// reproducible.
constexpr int kRows = 8;
constexpr int kGroup = 8;
constexpr int kDotWaves = 4;  // waves per work-group of k_dots_part
__global__ void __launch_bounds__(64 * kDotWaves)
    k_dots_part(const double2 *V, const double2 *w, int64_t ld, int64_t vstride, int64_t lo,
                int64_t hi, int nv, int sys0, int S, int64_t np_stride, double2 *part) {
  const int r = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * kDotWaves + (threadIdx.x >> 6);
  double2 wv[kRows];
  int64_t idx[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    idx[k] = lo + ((int64_t)blockIdx.x * kRows + k) * blockDim.x + threadIdx.x;
    wv[k] = idx[k] < hi ? w[(int64_t)r * ld + idx[k]] : make_double2(0.0, 0.0);
  }
  const int i1 = min(nv, (int)(blockIdx.z + 1) * kGroup);
  for (int i = blockIdx.z * kGroup; i < i1; ++i) {
    const double2 *v = V + (int64_t)i * vstride + (int64_t)r * ld;
    double a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      if (idx[k] < hi) {
        const double2 q = v[idx[k]];
        a += q.x * wv[k].x + q.y * wv[k].y;
        b += q.x * wv[k].y - q.y * wv[k].x;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    if (lane == 0) part[((int64_t)i * S + sys0 + r) * np_stride + p] = make_double2(a, b);
  }
}
// partials per work-group of k_dots_part over n rows
int64_t dot_parts(int64_t n) { return (n + 64 * kDotWaves * kRows - 1) / (64 * kDotWaves * kRows) * kDotWaves; }

// out[i S + s] = sum_{p < np} part[(i S + s) np_stride + p], fixed order;
// one wave per (i, s): blockIdx.x = i, blockIdx.y = s - sys0
__global__ void __launch_bounds__(64)
    k_part_reduce(const double2 *part, int64_t np_stride, int np, int sys0, int S, double2 *out) {
  const int64_t row = (int64_t)blockIdx.x * S + sys0 + blockIdx.y;
  const double2 *pp = part + row * np_stride;
  double a = 0, b = 0;
  for (int q = threadIdx.x; q < np; q += 64) {
    a += pp[q].x;
    b += pp[q].y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if (threadIdx.x == 0) out[row] = make_double2(a, b);
}

// w[r][row] -= sum_{i<nv} h[i*S + s] V[i][r][row]
__global__ void k_sub_basis(const double2 *V, double2 *w, int64_t ld, int64_t vstride, int64_t lo,
                            int64_t hi, int nv, int sys0, int S, const double2 *h) {
  const int r = blockIdx.y;
  const int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= hi) return;
  double2 acc = w[(int64_t)r * ld + n];
  for (int i = 0; i < nv; ++i) {
    const double2 c = h[(int64_t)i * S + sys0 + r];
    const double2 p = V[(int64_t)i * vstride + (int64_t)r * ld + n];
    acc.x -= c.x * p.x - c.y * p.y;
    acc.y -= c.x * p.y + c.y * p.x;
  }
  w[(int64_t)r * ld + n] = acc;
}

// part[s kNormParts + blockIdx.x] = sum |w|^2 over the block's rows of system
// s (grid-stride); k_norm_reduce adds the partials in a fixed order
constexpr int kNormParts = 1024;  // upper bound of the grid's x extent
__global__ void __launch_bounds__(kRed)
    k_norm2_part(const double2 *w, int64_t ld, int64_t lo, int64_t hi, int sys0, double *part) {
  const int r = blockIdx.y;
  double a = 0;
  for (int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < hi;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double2 p = w[(int64_t)r * ld + n];
    a += p.x * p.x + p.y * p.y;
  }
  const double2 t = block_sum2(a, 0.0);
  if (threadIdx.x == 0) part[(int64_t)(sys0 + r) * kNormParts + blockIdx.x] = t.x;
}
__global__ void __launch_bounds__(64)
    k_norm_reduce(const double *part, int np, int sys0, double *nrm) {
  const int s = sys0 + blockIdx.x;
  double a = 0;
  for (int q = threadIdx.x; q < np; q += 64) a += part[(int64_t)s * kNormParts + q];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if (threadIdx.x == 0) nrm[s] = a;
}

// out[r][row] = w[r][row] / sqrt(nrm[s]) (0 if nrm == 0)
__global__ void k_normalize(const double2 *w, double2 *out, int64_t ld, int64_t lo, int64_t hi,
                            int sys0, const double *nrm) {
  const int r = blockIdx.y;
  const int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= hi) return;
  const double s = nrm[sys0 + r];
  const double inv = s > 0 ? 1.0 / sqrt(s) : 0.0;
  const double2 p = w[(int64_t)r * ld + n];
  out[(int64_t)r * ld + n] = make_double2(p.x * inv, p.y * inv);
}

// The end of an Arnoldi step in one launch: the squared norm of w from the
// k_norm2_part partials (every work-group adds them in the order of
// k_norm_reduce; work-group 0 stores it for the Givens kernel), v_{j+1} =
// w / |w| into out, and the next step's preconditioned vector
// z = dinv v_{j+1} (what k_precond would compute from out).
__global__ void __launch_bounds__(256)
    k_normalize_next(const double2 *w, double2 *out, double2 *z, const double2 *dinv, int64_t ld,
                     int64_t lo, int64_t hi, int sys0, const double *part, int np, double *nrm) {
  __shared__ double snrm;
  const int r = blockIdx.y;
  const int s = sys0 + r;
  if (threadIdx.x < 64) {
    double a = 0;
    for (int q = threadIdx.x; q < np; q += 64) a += part[(int64_t)s * kNormParts + q];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (threadIdx.x == 0) {
      snrm = a;
      if (blockIdx.x == 0) nrm[s] = a;
    }
  }
  __syncthreads();
  const int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= hi) return;
  const double sv = snrm;
  const double inv = sv > 0 ? 1.0 / sqrt(sv) : 0.0;
  const double2 p = w[(int64_t)r * ld + n];
  const double2 v = make_double2(p.x * inv, p.y * inv);
  out[(int64_t)r * ld + n] = v;
  const double2 d = dinv[n];
  z[(int64_t)r * ld + n] = make_double2(v.x * d.x - v.y * d.y, v.x * d.y + v.y * d.x);
}

// z[r][row] = v[r][row] / d[row]
__global__ void k_precond(const double2 *v, double2 *z, const double2 *dinv, int64_t ld, int R) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ld) return;
  const double2 d = dinv[n];
  for (int r = 0; r < R; ++r) {
    const double2 p = v[(int64_t)r * ld + n];
    z[(int64_t)r * ld + n] = make_double2(p.x * d.x - p.y * d.y, p.x * d.y + p.y * d.x);
  }
}

// x[r][row] += dinv[row] * sum_i y[i*S + s] V[i][r][row]
__global__ void k_update_x(const double2 *V, double2 *x, const double2 *dinv, int64_t ld,
                           int64_t vstride, int64_t lo, int64_t hi, int nv_max, const int *nv_sys,
                           int sys0, int S, const double2 *y) {
  const int r = blockIdx.y;
  const int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= hi) return;
  const int nv = min(nv_max, nv_sys[sys0 + r]);
  double ax = 0, ay = 0;
  for (int i = 0; i < nv; ++i) {
    const double2 c = y[(int64_t)i * S + sys0 + r];
    const double2 p = V[(int64_t)i * vstride + (int64_t)r * ld + n];
    ax += c.x * p.x - c.y * p.y;
    ay += c.x * p.y + c.y * p.x;
  }
  const double2 d = dinv[n];
  double2 xv = x[(int64_t)r * ld + n];
  xv.x += ax * d.x - ay * d.y;
  xv.y += ax * d.y + ay * d.x;
  x[(int64_t)r * ld + n] = xv;
}

// r = b - r_in (in place on r: r = b - Ax)
__global__ void k_residual(const double2 *b, double2 *ax, int64_t count) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= count) return;
  const double2 p = b[n], q = ax[n];
  ax[n] = make_double2(p.x - q.x, p.y - q.y);
}

__global__ void k_axpy_real(double2 *x, const double2 *d, int64_t count) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= count) return;
  x[n].x += d[n].x;
  x[n].y += d[n].y;
}

__global__ void k_inv_diag(const double2 *zd, double2 *dinv, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 d = zd[i];
  const double m = d.x * d.x + d.y * d.y;
  dinv[i] = make_double2(d.x / m, -d.y / m);
}

unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
unsigned red_blocks(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kNormParts, (n + kRed - 1) / kRed));
}

struct Ctx {
  Plan *pl;
  hipStream_t s;
  int R;  // right-hand sides per mesh
  int S;  // systems = nmesh * R
  int64_t ld;
  double2 *dinv;
  // meshes with a system still iterating: the Arnoldi steps skip the others'
  // products and Gram-Schmidt work (their systems are inactive, so nothing
  // reads what those steps would have written); empty = every mesh
  std::vector<char> on;
  bool mesh_on(int mi) const { return on.empty() || on[mi]; }
};

// y = A x with the operator of the given precision on c128 vectors
void apply(Ctx &c, aim_precision prec, const double2 *x, double2 *y) {
  matvec_plan(c.pl, prec == AIM_FP64 ? AIM_FP64 : AIM_MIXED_IO64, c.R, x, y, c.s, nullptr,
              c.on.empty() ? nullptr : &c.on);
}

// nrm[s] = |v_s|^2 for every system, on the device (partials, fixed order)
void norms_dev(Ctx &c, const double2 *v, double *part, double *nrm) {
  int mi = 0;
  for (auto &md : c.pl->mesh) {
    const unsigned nb = red_blocks(md.hp.n);
    hipLaunchKernelGGL(k_norm2_part, dim3(nb, c.R), dim3(kRed), 0, c.s, v, c.ld, md.offset,
                       md.offset + md.hp.n, mi * c.R, part);
    LAUNCHCHECK();
    hipLaunchKernelGGL(k_norm_reduce, dim3(c.R), dim3(64), 0, c.s, part, (int)nb, mi * c.R, nrm);
    LAUNCHCHECK();
    ++mi;
  }
}
// per-system squared norms of v (host result)
void norms(Ctx &c, const double2 *v, double *part, double *nrm, std::vector<double> &out) {
  norms_dev(c, v, part, nrm);
  out.resize(c.S);
  HIPCHECK(hipMemcpyAsync(out.data(), nrm, sizeof(double) * c.S, hipMemcpyDeviceToHost, c.s));
  HIPCHECK(hipStreamSynchronize(c.s));
}

// ---- device-side Givens rotations and back substitution (one thread per
// system). Complex values as double2.
__device__ inline double2 cmul_(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconjmul_(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

struct GmresDev {
  double2 *H;      // [S][(m+1) m], column j of system s at H[s][i*m + j]
  double2 *cs, *sn;  // [S][m]
  double2 *g;      // [S][m+1]
  int *active;     // [S]
  int *its;        // [S] iterations counted
  int *jend;       // [S] columns of the current cycle
  double *tol_abs;  // [S] stop when |g_{j+1}| <= tol_abs
};

// New Hessenberg column j of every active system (one 64-lane work-group per
// system): sum of the two Gram-Schmidt passes and the norm; apply the
// previous rotations, form the new one, update the residual estimate
// |g_{j+1}|. The column and the rotations are staged in LDS by all lanes; the
// rotation chain itself is sequential. LDS: (3m + 1) complex values.
__global__ void __launch_bounds__(64)
    k_givens(GmresDev d, const double2 *h1, const double2 *h2, const double *nrm, int j, int m,
             int S) {
  const int s = blockIdx.x;
  if (!d.active[s]) return;  // uniform over the work-group
  extern __shared__ double2 gsh[];
  double2 *col = gsh, *cl = gsh + (m + 1), *sl = cl + m;
  double2 *Hs = d.H + (int64_t)s * (m + 1) * m;
  double2 *cs = d.cs + (int64_t)s * m, *sn = d.sn + (int64_t)s * m;
  for (int i = threadIdx.x; i <= j; i += 64) {
    const double2 a = h1[(int64_t)i * S + s], b = h2[(int64_t)i * S + s];
    col[i] = make_double2(a.x + b.x, a.y + b.y);
  }
  for (int i = threadIdx.x; i < j; i += 64) {
    cl[i] = cs[i];
    sl[i] = sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 *g = d.g + (int64_t)s * (m + 1);
    const double2 hj1 = make_double2(sqrt(nrm[s]), 0.0);
    for (int i = 0; i < j; ++i) {
      const double2 hi = col[i], hn = col[i + 1];
      // [hi; hn] <- [conj(c) hi + conj(s) hn; -s hi + c hn]
      const double2 t0 = cconjmul_(cl[i], hi), t1 = cconjmul_(sl[i], hn);
      const double2 u0 = cmul_(sl[i], hi), u1 = cmul_(cl[i], hn);
      col[i] = make_double2(t0.x + t1.x, t0.y + t1.y);
      col[i + 1] = make_double2(u1.x - u0.x, u1.y - u0.y);
    }
    const double2 a = col[j];
    const double den = sqrt(a.x * a.x + a.y * a.y + hj1.x * hj1.x);
    double2 c, sv;
    if (den == 0.0) {
      c = make_double2(1.0, 0.0);
      sv = make_double2(0.0, 0.0);
    } else {
      c = make_double2(a.x / den, a.y / den);
      sv = make_double2(hj1.x / den, 0.0);
    }
    cs[j] = c;
    sn[j] = sv;
    col[j] = make_double2(den, 0.0);
    col[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = g[j];
    const double2 gn = cmul_(sv, gj);
    g[j + 1] = make_double2(-gn.x, -gn.y);
    g[j] = cconjmul_(c, gj);
    d.its[s] += 1;
    d.jend[s] = j + 1;
    const double res = sqrt(gn.x * gn.x + gn.y * gn.y);
    if (res <= d.tol_abs[s] || den == 0.0) d.active[s] = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += 64) Hs[i * m + j] = col[i];
}

// y = H^-1 g on the jend x jend upper triangle (y stored [i][s] like h); one
// 64-lane work-group per system: rows bottom-up, each row's sum over the
// known y_k split over the lanes (fixed order). LDS: m complex values.
__global__ void __launch_bounds__(64) k_backsub(GmresDev d, double2 *y, int m, int S) {
  const int s = blockIdx.x;
  extern __shared__ double2 ysh[];
  const int n = d.jend[s];
  const double2 *Hs = d.H + (int64_t)s * (m + 1) * m;
  const double2 *g = d.g + (int64_t)s * (m + 1);
  for (int i = n - 1; i >= 0; --i) {
    double ax = 0, ay = 0;
    for (int k = i + 1 + threadIdx.x; k < n; k += 64) {
      const double2 t = cmul_(Hs[i * m + k], ysh[k]);
      ax += t.x;
      ay += t.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
      ax += __shfl_xor(ax, off, 64);
      ay += __shfl_xor(ay, off, 64);
    }
    if (threadIdx.x == 0) {
      const double2 gi = g[i];
      const double2 acc = make_double2(gi.x - ax, gi.y - ay);
      const double2 hd = Hs[i * m + i];
      const double dd = hd.x * hd.x + hd.y * hd.y;
      ysh[i] = dd == 0.0 ? make_double2(0.0, 0.0)
                         : make_double2((acc.x * hd.x + acc.y * hd.y) / dd,
                                        (acc.y * hd.x - acc.x * hd.y) / dd);
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += 64) y[(int64_t)i * S + s] = ysh[i];
}

struct Work {
  double2 *V = nullptr;  // (m+1) x R x ld
  double2 *z = nullptr, *w = nullptr;
  double2 *h1 = nullptr, *h2 = nullptr, *y = nullptr;
  double *nrm = nullptr;
  double2 *part = nullptr;  // dot-product partials [(m+1) S][np_stride]
  int64_t np_stride = 0;
  double *npart = nullptr;  // norm partials [S][kNormParts]
  GmresDev dev{};
};

constexpr int kCheckEvery = 8;  // iterations between convergence checks on the host

}  // namespace

// Buffers, stream and captured graphs of the solver, kept in the plan for
// the shape (right-hand sides per mesh R, restart m) of the last solve.
struct SolverState {
  int R = 0, m = 0;
  Work wk;
  double2 *dinv = nullptr;  // Jacobi: 1 / diag(Z^MOM)
  std::vector<void *> bufs;
  hipStream_t stream = nullptr;
  hipEvent_t entry = nullptr;
  // (precision, j0, j1, meshes still iterating as bits)
  std::map<std::tuple<int, int, int, uint32_t>, hipGraphExec_t> graphs;
  uint64_t gen = 0;       // plan work-buffer generation the graphs were captured with
  bool warm[2] = {false, false};  // a direct step of this precision ran on these buffers
};

namespace {

void drop_graphs(SolverState &st) {
  for (auto &g : st.graphs) (void)hipGraphExecDestroy(g.second);
  st.graphs.clear();
}

SolverState &solver_state(Plan *pl, int R, int m) {
  if (!pl->solver) pl->solver = new SolverState();
  SolverState &st = *pl->solver;
  if (!st.stream) {
    HIPCHECK(hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&st.entry, hipEventDisableTiming));
  }
  if (st.R == R && st.m == m) return st;
  HIPCHECK(hipStreamSynchronize(st.stream));
  drop_graphs(st);
  for (void *p : st.bufs) dev_free(pl, p);
  st.bufs.clear();
  st.R = st.m = 0;
  st.warm[0] = st.warm[1] = false;
  auto alloc = [&](size_t bytes) {
    void *p = dev_alloc(pl, bytes);
    st.bufs.push_back(p);
    return p;
  };
  const int S = pl->nmesh * R;
  const int64_t ld = pl->n_total, cnt = (int64_t)R * ld;
  Work &wk = st.wk;
  wk.V = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * cnt);
  wk.z = (double2 *)alloc(sizeof(double2) * cnt);
  wk.w = (double2 *)alloc(sizeof(double2) * cnt);
  wk.h1 = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S);
  wk.h2 = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S);
  wk.y = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S);
  wk.nrm = (double *)alloc(sizeof(double) * S);
  wk.np_stride = 0;
  for (auto &md : pl->mesh) wk.np_stride = std::max(wk.np_stride, dot_parts(md.hp.n));
  wk.part = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S * wk.np_stride);
  wk.npart = (double *)alloc(sizeof(double) * (size_t)S * kNormParts);
  wk.dev.H = (double2 *)alloc(sizeof(double2) * (size_t)S * (m + 1) * m);
  wk.dev.cs = (double2 *)alloc(sizeof(double2) * (size_t)S * m);
  wk.dev.sn = (double2 *)alloc(sizeof(double2) * (size_t)S * m);
  wk.dev.g = (double2 *)alloc(sizeof(double2) * (size_t)S * (m + 1));
  wk.dev.active = (int *)alloc(sizeof(int) * S);
  wk.dev.its = (int *)alloc(sizeof(int) * S);
  wk.dev.jend = (int *)alloc(sizeof(int) * S);
  wk.dev.tol_abs = (double *)alloc(sizeof(double) * S);
  st.dinv = (double2 *)alloc(sizeof(double2) * ld);
  for (auto &md : pl->mesh) {
    hipLaunchKernelGGL(k_inv_diag, dim3(nblk(md.hp.n, 256)), dim3(256), 0, st.stream, md.zdiag,
                       st.dinv + md.offset, md.hp.n);
    LAUNCHCHECK();
  }
  st.R = R;
  st.m = m;
  return st;
}

// One Arnoldi step j of every system: w = A D^-1 V[j], two classical
// Gram-Schmidt passes, V[j+1] = w / |w|, Hessenberg column j and rotation.
void arnoldi_step(Ctx &c, aim_precision prec, Work &wk, int j, int m) {
  const int S = c.S, R = c.R;
  const int64_t ld = c.ld, vstride = (int64_t)R * ld;
  if (j == 0) {  // later steps find z = dinv v_j left by the previous step
    hipLaunchKernelGGL(k_precond, dim3(nblk(ld, 256)), dim3(256), 0, c.s, wk.V + j * vstride, wk.z,
                       c.dinv, ld, R);
    LAUNCHCHECK();
  }
  apply(c, prec, wk.z, wk.w);
  for (int pass = 0; pass < 2; ++pass) {
    double2 *h = pass == 0 ? wk.h1 : wk.h2;
    int mi = 0;
    for (auto &md : c.pl->mesh) {
      if (!c.mesh_on(mi)) {
        ++mi;
        continue;
      }
      const int64_t nb = dot_parts(md.hp.n) / kDotWaves;
      hipLaunchKernelGGL(k_dots_part, dim3((unsigned)nb, R, nblk(j + 1, kGroup)),
                         dim3(64 * kDotWaves), 0, c.s, wk.V, wk.w, ld, vstride, md.offset,
                         md.offset + md.hp.n, j + 1, mi * R, S, wk.np_stride, wk.part);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_part_reduce, dim3(j + 1, R), dim3(64), 0, c.s, wk.part, wk.np_stride,
                         (int)(nb * kDotWaves), mi * R, S, h);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_sub_basis, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.V, wk.w,
                         ld, vstride, md.offset, md.offset + md.hp.n, j + 1, mi * R, S, h);
      LAUNCHCHECK();
      ++mi;
    }
  }
  int mi = 0;
  for (auto &md : c.pl->mesh) {
    if (!c.mesh_on(mi)) {
      ++mi;
      continue;
    }
    const unsigned nb = red_blocks(md.hp.n);
    hipLaunchKernelGGL(k_norm2_part, dim3(nb, R), dim3(kRed), 0, c.s, wk.w, ld, md.offset,
                       md.offset + md.hp.n, mi * R, wk.npart);
    LAUNCHCHECK();
    hipLaunchKernelGGL(k_normalize_next, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.w,
                       wk.V + (j + 1) * vstride, wk.z, c.dinv, ld, md.offset, md.offset + md.hp.n,
                       mi * R, wk.npart, (int)nb, wk.nrm);
    LAUNCHCHECK();
    ++mi;
  }
  hipLaunchKernelGGL(k_givens, dim3(S), dim3(64), sizeof(double2) * (3 * (size_t)m + 1), c.s,
                     wk.dev, wk.h1, wk.h2, wk.nrm, j, m, S);
  LAUNCHCHECK();
}

// Steps j0 .. j1-1 as one HIP graph: captured on first use, replayed after.
void run_segment_graph(Plan *pl, SolverState &st, Ctx &c, aim_precision prec, int j0, int j1) {
  if (pl->work_gen != st.gen) {  // a grid work buffer moved since the capture
    drop_graphs(st);
    st.gen = pl->work_gen;
  }
  uint32_t bits = 0;
  for (int i = 0; i < c.pl->nmesh; ++i)
    if (c.mesh_on(i)) bits |= 1u << i;
  const auto key = std::make_tuple((int)prec, j0, j1, bits);
  auto it = st.graphs.find(key);
  if (it == st.graphs.end()) {
    HIPCHECK(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      for (int j = j0; j < j1; ++j) arnoldi_step(c, prec, st.wk, j, st.m);
    } catch (...) {
      (void)hipStreamEndCapture(c.s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHECK(hipStreamEndCapture(c.s, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHECK(e);
    it = st.graphs.emplace(key, ex).first;
  }
  HIPCHECK(hipGraphLaunch(it->second, c.s));
}

// Solve A d = rhs (d starts at 0) for every system to a relative residual
// tol_s (estimated by the Arnoldi recurrence), restarted every m steps; a
// low-precision run also stops a system whose true residual has reached the
// operator's rounding floor (see the restart check). The
// Arnoldi step, the rotations and the residual estimate stay on the device;
// the host reads the active flags every kCheckEvery iterations. Returns the
// iterations used (lock-step count); `its` per system, `nprod` products.
int gmres_run(Ctx &c, SolverState &st, aim_precision prec, bool graphs, const double2 *rhs,
              double2 *d, const std::vector<double> &rhs_norm2, const std::vector<double> &tol_s,
              int max_iter, std::vector<int> &its, int &nprod) {
  Work &wk = st.wk;
  const int m = st.m;
  const int S = c.S, R = c.R;
  const int64_t ld = c.ld, vstride = (int64_t)R * ld, cnt = vstride;
  const int pi = prec == AIM_FP64 ? 0 : 1;
  HIPCHECK(hipMemsetAsync(d, 0, sizeof(double2) * cnt, c.s));
  std::vector<char> done(S, 0);
  for (int s = 0; s < S; ++s)
    if (rhs_norm2[s] == 0.0) done[s] = 1;
  int total = 0;
  std::vector<double> r2, prev(S, 0.0);
  bool first_cycle = true;
  std::vector<int> act(S), itd(S), jendh(S, m);
  HIPCHECK(hipMemcpyAsync(wk.dev.its, its.data(), sizeof(int) * S, hipMemcpyHostToDevice, c.s));
  // meshes with a system for which flag[s] is set
  auto meshes_of = [&](const auto &flag) {
    std::vector<char> on(c.pl->nmesh, 0);
    for (int s = 0; s < S; ++s)
      if (flag[s]) on[s / R] = 1;
    return on;
  };
  std::vector<char> notdone(S);
  while (true) {
    for (int s = 0; s < S; ++s) notdone[s] = !done[s];
    c.on = meshes_of(notdone);
    // residual of the current iterate: r = rhs - A d (rhs itself on the first cycle)
    if (first_cycle) {
      HIPCHECK(hipMemcpyAsync(wk.w, rhs, sizeof(double2) * cnt, hipMemcpyDeviceToDevice, c.s));
    } else {
      apply(c, prec, d, wk.w);
      ++nprod;
      hipLaunchKernelGGL(k_residual, dim3(nblk(cnt, 256)), dim3(256), 0, c.s, rhs, wk.w, cnt);
      LAUNCHCHECK();
    }
    const bool restarted = !first_cycle;
    first_cycle = false;
    norms(c, wk.w, wk.npart, wk.nrm, r2);
    bool all = true;
    for (int s = 0; s < S; ++s) {
      if (!done[s] && r2[s] <= tol_s[s] * tol_s[s] * rhs_norm2[s]) done[s] = 1;
      // Low-precision operator at its rounding floor: the last cycle's
      // estimate met the tolerance before the restart length, yet the true
      // residual of this operator did not even halve. Further cycles only
      // chase rounding noise; the FP64 refinement around this run continues.
      if (!done[s] && restarted && prec != AIM_FP64 && jendh[s] < m && r2[s] > 0.25 * prev[s])
        done[s] = 1;
      prev[s] = r2[s];
      all &= (bool)done[s];
    }
    if (all || total >= max_iter) break;
    // V[0] = r / |r|; cycle state on the device
    {
      int mi = 0;
      for (auto &md : c.pl->mesh) {
        hipLaunchKernelGGL(k_normalize, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.w, wk.V,
                           ld, md.offset, md.offset + md.hp.n, mi * R, wk.nrm);
        LAUNCHCHECK();
        ++mi;
      }
    }
    std::vector<double2> g0((size_t)S * (m + 1), make_double2(0, 0));
    std::vector<double> tabs(S);
    for (int s = 0; s < S; ++s) {
      act[s] = !done[s];
      g0[(size_t)s * (m + 1)] = make_double2(std::sqrt(r2[s]), 0.0);
      tabs[s] = tol_s[s] * std::sqrt(rhs_norm2[s]);
    }
    std::vector<int> zero(S, 0);
    HIPCHECK(hipMemcpyAsync(wk.dev.g, g0.data(), sizeof(double2) * g0.size(), hipMemcpyHostToDevice, c.s));
    HIPCHECK(hipMemcpyAsync(wk.dev.active, act.data(), sizeof(int) * S, hipMemcpyHostToDevice, c.s));
    HIPCHECK(hipMemcpyAsync(wk.dev.tol_abs, tabs.data(), sizeof(double) * S, hipMemcpyHostToDevice, c.s));
    HIPCHECK(hipMemcpyAsync(wk.dev.jend, zero.data(), sizeof(int) * S, hipMemcpyHostToDevice, c.s));
    // segments of kCheckEvery steps between polls of the active flags; a full
    // segment (or the cycle's last) is a graph once this precision has run
    // directly on the current buffers (so no buffer is allocated in a capture)
    c.on = meshes_of(act);
    for (int j = 0; j < m && total < max_iter;) {
      const int j1 = std::min({j + kCheckEvery, m, j + (max_iter - total)});
      const bool whole = (j1 - j == kCheckEvery) || j1 == m;
      if (graphs && whole && st.warm[pi]) {
        run_segment_graph(c.pl, st, c, prec, j, j1);
      } else {
        for (int jj = j; jj < j1; ++jj) arnoldi_step(c, prec, wk, jj, m);
        st.warm[pi] = true;
      }
      nprod += j1 - j;
      total += j1 - j;
      j = j1;
      HIPCHECK(hipMemcpyAsync(act.data(), wk.dev.active, sizeof(int) * S, hipMemcpyDeviceToHost, c.s));
      HIPCHECK(hipStreamSynchronize(c.s));
      bool any = false;
      for (int s = 0; s < S; ++s) any |= (bool)act[s];
      if (!any) break;
      c.on = meshes_of(act);
    }
    // d += D^-1 V y, y = H^-1 g per system (systems done before the cycle: jend = 0)
    hipLaunchKernelGGL(k_backsub, dim3(S), dim3(64), sizeof(double2) * (size_t)m, c.s, wk.dev,
                       wk.y, m, S);
    LAUNCHCHECK();
    {
      int mi = 0;
      for (auto &md : c.pl->mesh) {
        hipLaunchKernelGGL(k_update_x, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.V, d,
                           c.dinv, ld, vstride, md.offset, md.offset + md.hp.n, m, wk.dev.jend,
                           mi * R, S, wk.y);
        LAUNCHCHECK();
        ++mi;
      }
    }
    HIPCHECK(hipMemcpyAsync(jendh.data(), wk.dev.jend, sizeof(int) * S, hipMemcpyDeviceToHost, c.s));
    HIPCHECK(hipStreamSynchronize(c.s));
  }
  HIPCHECK(hipMemcpyAsync(itd.data(), wk.dev.its, sizeof(int) * S, hipMemcpyDeviceToHost, c.s));
  HIPCHECK(hipStreamSynchronize(c.s));
  for (int s = 0; s < S; ++s) its[s] = itd[s];
  c.on.clear();  // later products (the outer residual) cover every mesh
  return total;
}

}  // namespace

void solver_release(Plan *pl) {
  if (!pl || !pl->solver) return;
  SolverState &st = *pl->solver;
  if (st.stream) (void)hipStreamSynchronize(st.stream);
  drop_graphs(st);
  for (void *p : st.bufs) dev_free(pl, p);
  if (st.entry) (void)hipEventDestroy(st.entry);
  if (st.stream) (void)hipStreamDestroy(st.stream);
  delete pl->solver;
  pl->solver = nullptr;
}

aim_status gmres_solve(Plan *pl, aim_precision prec, int R, const aim_planewave *waves,
                       const aim_solve_opts &o, double2 *x, aim_solve_stats *st, hipStream_t caller) {
  auto t0 = std::chrono::steady_clock::now();
  const int S = pl->nmesh * R;
  const int m = o.restart;
  const int64_t ld = pl->n_total;
  const int64_t cnt = (int64_t)R * ld;
  const bool graphs = !(o.flags & AIM_SOLVE_NO_GRAPH);
  SolverState &ss = solver_state(pl, R, m);
  // the solve runs on the solver's own stream (capturable), after the
  // caller's stream has reached this call; it ends synchronised
  const hipStream_t s = ss.stream;
  HIPCHECK(hipEventRecord(ss.entry, caller));
  HIPCHECK(hipStreamWaitEvent(s, ss.entry, 0));
  Work &wk = ss.wk;
  std::vector<void *> tmp;
  auto alloc = [&](size_t bytes) {
    void *p = dev_alloc(pl, bytes);
    tmp.push_back(p);
    return p;
  };
  aim_status result = AIM_OK;
  try {
    double2 *b = (double2 *)alloc(sizeof(double2) * cnt);
    double2 *r = (double2 *)alloc(sizeof(double2) * cnt);
    double2 *dd = (double2 *)alloc(sizeof(double2) * cnt);
    for (auto &md : pl->mesh) excitation_mesh(pl, md, R, waves, b + md.offset, ld, s);
    Ctx c{pl, s, R, S, ld, ss.dinv};
    std::vector<double> b2, r2;
    norms(c, b, wk.npart, wk.nrm, b2);
    if (!o.warm_start) HIPCHECK(hipMemsetAsync(x, 0, sizeof(double2) * cnt, s));
    std::vector<int> its(S, 0);
    int n_low = 0, n64 = 0, total = 0;
    const double tol = o.tol;
    // residual r = b - A64 x
    auto residual = [&]() {
      apply(c, AIM_FP64, x, r);
      ++n64;
      hipLaunchKernelGGL(k_residual, dim3(nblk(cnt, 256)), dim3(256), 0, s, b, r, cnt);
      LAUNCHCHECK();
      norms(c, r, wk.npart, wk.nrm, r2);
    };
    if (prec == AIM_FP64) {
      if (o.warm_start) {
        residual();
      } else {
        HIPCHECK(hipMemcpyAsync(r, b, sizeof(double2) * cnt, hipMemcpyDeviceToDevice, s));
        r2 = b2;
      }
      std::vector<double> tol_s(S);
      for (int i = 0; i < S; ++i) tol_s[i] = r2[i] > 0 ? tol * std::sqrt(b2[i] / r2[i]) : 1.0;
      total += gmres_run(c, ss, AIM_FP64, graphs, r, dd, r2, tol_s, o.max_iter, its, n64);
      hipLaunchKernelGGL(k_axpy_real, dim3(nblk(cnt, 256)), dim3(256), 0, s, x, dd, cnt);
      LAUNCHCHECK();
      residual();
    } else {
      residual();
      for (int outer = 0; outer < 20; ++outer) {
        bool all = true;
        for (int i = 0; i < S; ++i) all &= (b2[i] == 0 || r2[i] <= tol * tol * b2[i]);
        if (all || total >= o.max_iter) break;
        std::vector<double> tol_s(S);
        for (int i = 0; i < S; ++i) {
          // reach the outer tolerance with margin, but not below what c64 arithmetic resolves
          double want = r2[i] > 0 ? 0.5 * tol * std::sqrt(b2[i] / r2[i]) : 1.0;
          tol_s[i] = std::max(want, 2e-6);
        }
        total += gmres_run(c, ss, AIM_MIXED, graphs, r, dd, r2, tol_s, o.max_iter - total, its,
                           n_low);
        hipLaunchKernelGGL(k_axpy_real, dim3(nblk(cnt, 256)), dim3(256), 0, s, x, dd, cnt);
        LAUNCHCHECK();
        residual();
      }
    }
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all_ok = true;
    for (int i = 0; i < S; ++i) {
      double rel = b2[i] > 0 ? std::sqrt(r2[i] / b2[i]) : 0.0;
      if (!(rel <= tol)) all_ok = false;
    }
    if (st) {  // one entry per system (mesh, wave), mesh-major
      for (int sidx = 0; sidx < S; ++sidx) {
        aim_solve_stats q{};
        const double rel = b2[sidx] > 0 ? std::sqrt(r2[sidx] / b2[sidx]) : 0.0;
        q.iterations = its[sidx];
        q.residual = rel;
        q.converged = rel <= tol ? 1 : 0;
        q.matvec_low = n_low;
        q.matvec_fp64 = n64;
        q.seconds = secs;
        st[sidx] = q;
      }
    }
    result = all_ok ? AIM_OK : AIM_ERR_NOCONV;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    for (void *p : tmp) dev_free(pl, p);
    throw;
  }
  HIPCHECK(hipStreamSynchronize(s));
  for (void *p : tmp) dev_free(pl, p);
  return result;
}

}  // namespace aim
