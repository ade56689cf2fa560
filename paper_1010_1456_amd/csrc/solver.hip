// Restarted GMRES with right Jacobi preconditioning (the matvec's caller).
//
// The paper solves with a diagonal preconditioner and stops on the relative
// RMS residual (Section 2.2). Here every (mesh, plane wave) pair is its own
// system; all systems advance in lock-step so one batched AIM product serves
// them all. Arnoldi runs in FP64 on the device (classical Gram-Schmidt, two
// passes); only the new Hessenberg column crosses to the host per iteration,
// where the Givens rotations and the convergence test run. For AIM_MIXED the
// inner solves use the c64 operator on c128 Krylov vectors, inside an FP64
// iterative-refinement loop r = b - A64 x that decides convergence.
#include <chrono>
#include <cmath>
#include <complex>

#include "aim_internal.h"

namespace aim {

namespace {

using zc = std::complex<double>;

constexpr int kRed = 256;

__device__ inline void atomic_add2(double2 *p, double a, double b) {
  unsafeAtomicAdd(&p->x, a);
  unsafeAtomicAdd(&p->y, b);
}

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

// h[i*S + s] += sum_rows conj(V[i][r][row]) w[r][row], s = sys0 + r
__global__ void __launch_bounds__(kRed)
    k_dots(const double2 *V, const double2 *w, int64_t ld, int64_t vstride, int64_t lo, int64_t hi,
           int sys0, int S, double2 *h) {
  const int i = blockIdx.y, r = blockIdx.z;
  const double2 *v = V + (int64_t)i * vstride + (int64_t)r * ld;
  const double2 *ww = w + (int64_t)r * ld;
  double a = 0, b = 0;
  for (int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < hi;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double2 p = v[n], q = ww[n];
    a += p.x * q.x + p.y * q.y;
    b += p.x * q.y - p.y * q.x;
  }
  const double2 t = block_sum2(a, b);
  if (threadIdx.x == 0) atomic_add2(&h[(int64_t)i * S + sys0 + r], t.x, t.y);
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

// nrm[s] += sum |w|^2 over the rows of system s
__global__ void __launch_bounds__(kRed)
    k_norm2(const double2 *w, int64_t ld, int64_t lo, int64_t hi, int sys0, double *nrm) {
  const int r = blockIdx.y;
  double a = 0;
  for (int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < hi;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double2 p = w[(int64_t)r * ld + n];
    a += p.x * p.x + p.y * p.y;
  }
  const double2 t = block_sum2(a, 0.0);
  if (threadIdx.x == 0) unsafeAtomicAdd(&nrm[sys0 + r], t.x);
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
unsigned red_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (n + kRed - 1) / kRed)); }

struct Ctx {
  Plan *pl;
  hipStream_t s;
  int R;  // right-hand sides per mesh
  int S;  // systems = nmesh * R
  int64_t ld;
  double2 *dinv;
};

// y = A x with the operator of the given precision on c128 vectors
void apply(Ctx &c, aim_precision prec, const double2 *x, double2 *y) {
  for (auto &md : c.pl->mesh) {
    if (prec == AIM_FP64)
      matvec_mesh<double, double, double>(c.pl, md, c.R, x + md.offset, c.ld, y + md.offset, c.ld, c.s);
    else
      matvec_mesh<float, double, double>(c.pl, md, c.R, x + md.offset, c.ld, y + md.offset, c.ld, c.s);
  }
}

// per-system squared norms of v (host result)
void norms(Ctx &c, const double2 *v, double *dscratch, std::vector<double> &out) {
  HIPCHECK(hipMemsetAsync(dscratch, 0, sizeof(double) * c.S, c.s));
  int mi = 0;
  for (auto &md : c.pl->mesh) {
    hipLaunchKernelGGL(k_norm2, dim3(red_blocks(md.hp.n), c.R), dim3(kRed), 0, c.s, v, c.ld,
                       md.offset, md.offset + md.hp.n, mi * c.R, dscratch);
    LAUNCHCHECK();
    ++mi;
  }
  out.resize(c.S);
  HIPCHECK(hipMemcpyAsync(out.data(), dscratch, sizeof(double) * c.S, hipMemcpyDeviceToHost, c.s));
  HIPCHECK(hipStreamSynchronize(c.s));
}

struct Work {
  double2 *V = nullptr;  // (m+1) x R x ld
  double2 *z = nullptr, *w = nullptr;
  double2 *h1 = nullptr, *h2 = nullptr, *y = nullptr;
  double *nrm = nullptr;
  int *nv = nullptr;
};

// Solve A d = rhs (d starts at 0) for every system to a relative residual
// tol_s (estimated by the Arnoldi recurrence), restarted every m steps.
// Returns the inner iterations used; `its` per system, `low` counts products.
int gmres_run(Ctx &c, aim_precision prec, Work &wk, int m, const double2 *rhs, double2 *d,
              const std::vector<double> &rhs_norm2, const std::vector<double> &tol_s, int max_iter,
              std::vector<int> &its, int &nprod) {
  const int S = c.S, R = c.R;
  const int64_t ld = c.ld, vstride = (int64_t)R * ld, cnt = vstride;
  HIPCHECK(hipMemsetAsync(d, 0, sizeof(double2) * cnt, c.s));
  std::vector<char> done(S, 0);
  for (int s = 0; s < S; ++s)
    if (rhs_norm2[s] == 0.0) done[s] = 1;
  int total = 0;
  std::vector<double> r2;
  bool first_cycle = true;
  while (true) {
    // residual of the current iterate: r = rhs - A d (rhs itself on the first cycle)
    if (first_cycle) {
      HIPCHECK(hipMemcpyAsync(wk.w, rhs, sizeof(double2) * cnt, hipMemcpyDeviceToDevice, c.s));
    } else {
      apply(c, prec, d, wk.w);
      ++nprod;
      hipLaunchKernelGGL(k_residual, dim3(nblk(cnt, 256)), dim3(256), 0, c.s, rhs, wk.w, cnt);
      LAUNCHCHECK();
    }
    first_cycle = false;
    norms(c, wk.w, wk.nrm, r2);
    bool all = true;
    for (int s = 0; s < S; ++s) {
      if (!done[s] && r2[s] <= tol_s[s] * tol_s[s] * rhs_norm2[s]) done[s] = 1;
      all &= (bool)done[s];
    }
    if (all || total >= max_iter) return total;
    // V[0] = r / |r|
    {
      int mi = 0;
      for (auto &md : c.pl->mesh) {
        hipLaunchKernelGGL(k_normalize, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.w, wk.V,
                           ld, md.offset, md.offset + md.hp.n, mi * R, wk.nrm);
        LAUNCHCHECK();
        ++mi;
      }
    }
    std::vector<std::vector<zc>> H(S, std::vector<zc>((m + 1) * m, 0.0));
    std::vector<std::vector<zc>> cs(S, std::vector<zc>(m)), sn(S, std::vector<zc>(m));
    std::vector<std::vector<zc>> g(S, std::vector<zc>(m + 1, 0.0));
    std::vector<int> jend(S, 0);
    std::vector<char> active(S);
    for (int s = 0; s < S; ++s) {
      g[s][0] = std::sqrt(r2[s]);
      active[s] = !done[s];
    }
    std::vector<double2> hh1((size_t)(m + 1) * S), hh2((size_t)(m + 1) * S);
    std::vector<double> nn(S);
    for (int j = 0; j < m && total < max_iter; ++j) {
      // w = A D^-1 V[j]
      hipLaunchKernelGGL(k_precond, dim3(nblk(ld, 256)), dim3(256), 0, c.s, wk.V + j * vstride, wk.z,
                         c.dinv, ld, R);
      LAUNCHCHECK();
      apply(c, prec, wk.z, wk.w);
      ++nprod;
      ++total;
      // two passes of classical Gram-Schmidt
      for (int pass = 0; pass < 2; ++pass) {
        double2 *h = pass == 0 ? wk.h1 : wk.h2;
        HIPCHECK(hipMemsetAsync(h, 0, sizeof(double2) * (j + 1) * S, c.s));
        int mi = 0;
        for (auto &md : c.pl->mesh) {
          hipLaunchKernelGGL(k_dots, dim3(red_blocks(md.hp.n), j + 1, R), dim3(kRed), 0, c.s, wk.V,
                             wk.w, ld, vstride, md.offset, md.offset + md.hp.n, mi * R, S, h);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_sub_basis, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.V,
                             wk.w, ld, vstride, md.offset, md.offset + md.hp.n, j + 1, mi * R, S, h);
          LAUNCHCHECK();
          ++mi;
        }
      }
      HIPCHECK(hipMemsetAsync(wk.nrm, 0, sizeof(double) * S, c.s));
      {
        int mi = 0;
        for (auto &md : c.pl->mesh) {
          hipLaunchKernelGGL(k_norm2, dim3(red_blocks(md.hp.n), R), dim3(kRed), 0, c.s, wk.w, ld,
                             md.offset, md.offset + md.hp.n, mi * R, wk.nrm);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_normalize, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.w,
                             wk.V + (j + 1) * vstride, ld, md.offset, md.offset + md.hp.n, mi * R,
                             wk.nrm);
          LAUNCHCHECK();
          ++mi;
        }
      }
      HIPCHECK(hipMemcpyAsync(hh1.data(), wk.h1, sizeof(double2) * (j + 1) * S, hipMemcpyDeviceToHost, c.s));
      HIPCHECK(hipMemcpyAsync(hh2.data(), wk.h2, sizeof(double2) * (j + 1) * S, hipMemcpyDeviceToHost, c.s));
      HIPCHECK(hipMemcpyAsync(nn.data(), wk.nrm, sizeof(double) * S, hipMemcpyDeviceToHost, c.s));
      HIPCHECK(hipStreamSynchronize(c.s));
      bool any_active = false;
      for (int s = 0; s < S; ++s) {
        if (!active[s]) continue;
        its[s]++;
        zc *Hc = &H[s][0];
        for (int i = 0; i <= j; ++i)
          Hc[i * m + j] = zc(hh1[(size_t)i * S + s].x + hh2[(size_t)i * S + s].x,
                             hh1[(size_t)i * S + s].y + hh2[(size_t)i * S + s].y);
        Hc[(j + 1) * m + j] = std::sqrt(nn[s]);
        for (int i = 0; i < j; ++i) {
          zc t = std::conj(cs[s][i]) * Hc[i * m + j] + std::conj(sn[s][i]) * Hc[(i + 1) * m + j];
          Hc[(i + 1) * m + j] = -sn[s][i] * Hc[i * m + j] + cs[s][i] * Hc[(i + 1) * m + j];
          Hc[i * m + j] = t;
        }
        zc a = Hc[j * m + j], b = Hc[(j + 1) * m + j];
        double den = std::sqrt(std::norm(a) + std::norm(b));
        if (den == 0) {
          cs[s][j] = 1;
          sn[s][j] = 0;
        } else {
          cs[s][j] = a / den;
          sn[s][j] = b / den;
        }
        Hc[j * m + j] = den;
        Hc[(j + 1) * m + j] = 0;
        g[s][j + 1] = -sn[s][j] * g[s][j];
        g[s][j] = std::conj(cs[s][j]) * g[s][j];
        jend[s] = j + 1;
        if (std::abs(g[s][j + 1]) <= tol_s[s] * std::sqrt(rhs_norm2[s]) || den == 0) active[s] = 0;
        any_active |= (bool)active[s];
      }
      if (!any_active) break;
    }
    // d += D^-1 V y, y = H^-1 g per system
    std::vector<double2> yv((size_t)m * S, make_double2(0, 0));
    std::vector<int> nv(S);
    int nv_max = 0;
    for (int s = 0; s < S; ++s) {
      const int n = done[s] ? 0 : jend[s];
      nv[s] = n;
      nv_max = std::max(nv_max, n);
      std::vector<zc> y(n);
      for (int i = n - 1; i >= 0; --i) {
        zc acc = g[s][i];
        for (int k = i + 1; k < n; ++k) acc -= H[s][i * m + k] * y[k];
        y[i] = H[s][i * m + i] == zc(0) ? zc(0) : acc / H[s][i * m + i];
      }
      for (int i = 0; i < n; ++i) yv[(size_t)i * S + s] = make_double2(y[i].real(), y[i].imag());
    }
    HIPCHECK(hipMemcpyAsync(wk.y, yv.data(), sizeof(double2) * m * S, hipMemcpyHostToDevice, c.s));
    HIPCHECK(hipMemcpyAsync(wk.nv, nv.data(), sizeof(int) * S, hipMemcpyHostToDevice, c.s));
    {
      int mi = 0;
      for (auto &md : c.pl->mesh) {
        hipLaunchKernelGGL(k_update_x, dim3(nblk(md.hp.n, 256), R), dim3(256), 0, c.s, wk.V, d,
                           c.dinv, ld, vstride, md.offset, md.offset + md.hp.n, nv_max, wk.nv,
                           mi * R, S, wk.y);
        LAUNCHCHECK();
        ++mi;
      }
    }
    HIPCHECK(hipStreamSynchronize(c.s));
  }
}

}  // namespace

aim_status gmres_solve(Plan *pl, aim_precision prec, int R, const aim_planewave *waves,
                       const aim_solve_opts &o, double2 *x, aim_solve_stats *st, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int S = pl->nmesh * R;
  const int m = o.restart;
  const int64_t ld = pl->n_total;
  const int64_t cnt = (int64_t)R * ld;
  std::vector<void *> tmp;
  auto alloc = [&](size_t bytes) {
    void *p = dev_alloc(pl, bytes);
    tmp.push_back(p);
    return p;
  };
  aim_status result = AIM_OK;
  try {
    Work wk;
    wk.V = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * cnt);
    wk.z = (double2 *)alloc(sizeof(double2) * cnt);
    wk.w = (double2 *)alloc(sizeof(double2) * cnt);
    wk.h1 = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S);
    wk.h2 = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S);
    wk.y = (double2 *)alloc(sizeof(double2) * (size_t)(m + 1) * S);
    wk.nrm = (double *)alloc(sizeof(double) * S);
    wk.nv = (int *)alloc(sizeof(int) * S);
    double2 *b = (double2 *)alloc(sizeof(double2) * cnt);
    double2 *r = (double2 *)alloc(sizeof(double2) * cnt);
    double2 *dd = (double2 *)alloc(sizeof(double2) * cnt);
    double2 *dinv = (double2 *)alloc(sizeof(double2) * ld);
    for (auto &md : pl->mesh) {
      hipLaunchKernelGGL(k_inv_diag, dim3(nblk(md.hp.n, 256)), dim3(256), 0, s, md.zdiag,
                         dinv + md.offset, md.hp.n);
      LAUNCHCHECK();
      excitation_mesh(pl, md, R, waves, b + md.offset, ld, s);
    }
    Ctx c{pl, s, R, S, ld, dinv};
    std::vector<double> b2, r2;
    norms(c, b, wk.nrm, b2);
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
      norms(c, r, wk.nrm, r2);
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
      total += gmres_run(c, AIM_FP64, wk, m, r, dd, r2, tol_s, o.max_iter, its, n64);
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
        total += gmres_run(c, AIM_MIXED, wk, m, r, dd, r2, tol_s, o.max_iter - total, its, n_low);
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
    if (st) {
      for (int w = 0; w < R; ++w) {
        aim_solve_stats q{};
        q.converged = 1;
        for (int mi = 0; mi < pl->nmesh; ++mi) {
          const int sidx = mi * R + w;
          double rel = b2[sidx] > 0 ? std::sqrt(r2[sidx] / b2[sidx]) : 0.0;
          q.iterations = std::max(q.iterations, its[sidx]);
          q.residual = std::max(q.residual, rel);
          if (!(rel <= tol)) q.converged = 0;
        }
        q.matvec_low = n_low;
        q.matvec_fp64 = n64;
        q.seconds = secs;
        st[w] = q;
      }
    }
    result = all_ok ? AIM_OK : AIM_ERR_NOCONV;
  } catch (...) {
    for (void *p : tmp) dev_free(pl, p);
    throw;
  }
  for (void *p : tmp) dev_free(pl, p);
  return result;
}

}  // namespace aim
