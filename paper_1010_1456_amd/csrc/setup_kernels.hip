// Operator set-up on the GPU (FP64): projection weights, grid Green's
// function spectrum, near-zone matrix, plane-wave right-hand sides.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "aim_internal.h"
#include "fft_map.h"
#include "geom_device.h"

namespace aim {
using namespace geo;

namespace {

__device__ inline void basis_side(const int32_t *rwg, const double *len, const double *area,
                                  const int32_t *tris, const double *verts, int64_t n, int side,
                                  D3 *T, double *A, D3 *free_v, double *s, double *l) {
  const int t = rwg[4 * n + side];
  const int fv = rwg[4 * n + 2 + side];
  for (int c = 0; c < 3; ++c) T[c] = vtx(verts, tris[3 * (int64_t)t + c]);
  *A = area[t];
  *free_v = vtx(verts, fv);
  *s = side == 0 ? 1.0 : -1.0;
  *l = len[n];
}

// Lambda[n][q][u] = sum_{T+-} A_T sum_p w_p F_q(r_p) l_u(r_p), q = x, y, z, div.
__global__ void k_projection(const int32_t *rwg, const double *len, const double *area,
                             const int32_t *tris, const double *verts, const int32_t *anchor3,
                             int64_t n, int M, double x0, double y0, double z0, double h,
                             double *lam) {
  const int K = (M + 1) * (M + 1) * (M + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t b = t / K;
  const int u = (int)(t - b * K);
  const int ui = u / ((M + 1) * (M + 1)), uj = (u / (M + 1)) % (M + 1), uk = u % (M + 1);
  const double ax = anchor3[3 * b], ay = anchor3[3 * b + 1], az = anchor3[3 * b + 2];
  double acc[4] = {0, 0, 0, 0};
  for (int side = 0; side < 2; ++side) {
    D3 T[3], pf;
    double A, s, l;
    basis_side(rwg, len, area, tris, verts, b, side, T, &A, &pf, &s, &l);
    const double cf = s * l / (2.0 * A);
    const double dv = s * l / A;
    for (int p = 0; p < 7; ++p) {
      double w;
      const D3 r = quad_point(T, p, &w);
      const double xi[3] = {(r.x - x0) / h - ax, (r.y - y0) / h - ay, (r.z - z0) / h - az};
      const int sel[3] = {ui, uj, uk};
      double lw = 1.0;
      for (int d = 0; d < 3; ++d) {
        double v = 1.0;
        for (int m = 0; m <= M; ++m)
          if (m != sel[d]) v *= (xi[d] - m) / (double)(sel[d] - m);
        lw *= v;
      }
      const double aw = A * w * lw;
      acc[0] += aw * cf * (r.x - pf.x);
      acc[1] += aw * cf * (r.y - pf.y);
      acc[2] += aw * cf * (r.z - pf.z);
      acc[3] += aw * dv;
    }
  }
  for (int q = 0; q < 4; ++q) lam[(b * 4 + q) * K + u] = acc[q];
}

// unit normal (v1 - v0) x (v2 - v0) of a triangle
__device__ inline D3 tri_normal(const D3 *T) {
  const D3 c = cross(T[1] - T[0], T[2] - T[0]);
  return (1.0 / norm(c)) * c;
}

// l_s(xi) and its derivative for the nodes 0..M
__device__ inline void lagrange_and_deriv(double xi, int s, int M, double *l, double *dl) {
  double v = 1.0, dv = 0.0;
  for (int m = 0; m <= M; ++m) {
    if (m == s) continue;
    const double f = 1.0 / (double)(s - m);
    dv = dv * (xi - m) * f + v * f;  // product rule, factor by factor
    v *= (xi - m) * f;
  }
  *l = v;
  *dl = dv;
}

// Curl weights of the combined field: W[n][e][u] = sum_{T+-} A_T sum_p w_p
// (t(r_p) x grad l_u(r_p))_e with t = f_n x n_T, so that sum_{e,u} W_e[u]
// A_e[u] = int t . curl A for the interpolant of a grid field A.
__global__ void k_curl_projection(const int32_t *rwg, const double *len, const double *area,
                                  const int32_t *tris, const double *verts, const int32_t *anchor3,
                                  int64_t n, int M, double x0, double y0, double z0, double h,
                                  double *curl) {
  const int K = (M + 1) * (M + 1) * (M + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t b = t / K;
  const int u = (int)(t - b * K);
  const int sel[3] = {u / ((M + 1) * (M + 1)), (u / (M + 1)) % (M + 1), u % (M + 1)};
  const double ax = anchor3[3 * b], ay = anchor3[3 * b + 1], az = anchor3[3 * b + 2];
  D3 acc = d3(0, 0, 0);
  for (int side = 0; side < 2; ++side) {
    D3 T[3], pf;
    double A, s, l;
    basis_side(rwg, len, area, tris, verts, b, side, T, &A, &pf, &s, &l);
    const D3 nt = tri_normal(T);
    const double cf = s * l / (2.0 * A);
    for (int p = 0; p < 7; ++p) {
      double w;
      const D3 r = quad_point(T, p, &w);
      const double xi[3] = {(r.x - x0) / h - ax, (r.y - y0) / h - ay, (r.z - z0) / h - az};
      double L[3], D[3];
      for (int d = 0; d < 3; ++d) lagrange_and_deriv(xi[d], sel[d], M, &L[d], &D[d]);
      const D3 g = (1.0 / h) * d3(D[0] * L[1] * L[2], L[0] * D[1] * L[2], L[0] * L[1] * D[2]);
      const D3 tv = cross(cf * (r - pf), nt);
      acc = acc + (A * w) * cross(tv, g);
    }
  }
  curl[(b * 3 + 0) * K + u] = acc.x;
  curl[(b * 3 + 1) * K + u] = acc.y;
  curl[(b * 3 + 2) * K + u] = acc.z;
}

// 1 where a (basis, stencil node) pair has any non-zero weight: projection
// or, for the combined field, curl weight (the node is then read by the
// interpolation even where its projection weights vanish, as off a flat face
// lying in a grid plane)
__global__ void k_lam_mask(const double *lam, const double *curl, int64_t n, int K,
                           uint8_t *mask) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t b = t / K;
  const int u = (int)(t - b * K);
  bool nz = false;
  for (int q = 0; q < 4; ++q) nz |= lam[(b * 4 + q) * K + u] != 0.0;
  if (curl)
    for (int e = 0; e < 3; ++e) nz |= curl[(b * 3 + e) * K + u] != 0.0;
  mask[t] = nz ? 1 : 0;
}

// lamT[e][q] = Lambda[src / K][q][src % K] for entry e with src = ent_src[e]
__global__ void k_lam_transpose(const double *lam, const int32_t *ent_src, int64_t ne, int K,
                                double *lamT64, float *lamT32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int64_t src = ent_src[e];
  const int64_t b = src / K;
  const int u = (int)(src - b * K);
  for (int q = 0; q < 4; ++q) {
    const double v = lam[(b * 4 + q) * K + u];
    lamT64[e * 4 + q] = v;
    if (lamT32) lamT32[e * 4 + q] = (float)v;
  }
}

__global__ void k_to_float(const double *in, float *out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__device__ inline double2 green(double k, double R) {
  if (R == 0.0) return make_double2(0.0, 0.0);
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double g = 0.25 / (3.14159265358979323846 * R);
  return make_double2(g * cs, -g * sn);
}

// g on the circulant embedding [Px][Py][Pz]: index i folds to min(i, P - i)
__global__ void k_embed_green(double2 *out, int Px, int Py, int Pz, int Nx, int Ny, int Nz,
                              double k, double h) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)Px * Py * Pz;
  if (t >= tot) return;
  const int kk = (int)(t % Pz);
  const int jj = (int)((t / Pz) % Py);
  const int ii = (int)(t / ((int64_t)Py * Pz));
  const int fi = min(ii, Px - ii), fj = min(jj, Py - jj), fk = min(kk, Pz - kk);
  double2 v = make_double2(0.0, 0.0);
  if (fi < Nx && fj < Ny && fk < Nz) {
    const double R = h * sqrt((double)fi * fi + (double)fj * fj + (double)fk * fk);
    v = green(k, R);
  }
  out[t] = v;
}

// z range of the grid planes holding a non-zero projection weight
__global__ void k_lam_zrange(const double *lam, const int32_t *anchor3, int64_t n, int M,
                             int *zr) {
  const int K = (M + 1) * (M + 1) * (M + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t b = t / K;
  const int u = (int)(t - b * K);
  bool nz = false;
  for (int q = 0; q < 4; ++q) nz |= lam[(b * 4 + q) * K + u] != 0.0;
  if (!nz) return;
  const int z = anchor3[3 * b + 2] + u % (M + 1);
  atomicMin(&zr[0], z);
  atomicMax(&zr[1], z);
}

// in-plane weights: plane_lam[b][q][ui (M+1) + uj] = lam[b][q][u] with u's
// z index on the plane
__global__ void k_lam_plane(const double *lam, const int32_t *anchor3, int64_t n, int M, int zp,
                            double *plane_lam) {
  const int K = (M + 1) * (M + 1) * (M + 1), K2 = (M + 1) * (M + 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K2) return;
  const int64_t b = t / K2;
  const int u2 = (int)(t - b * K2);
  const int uk = zp - anchor3[3 * b + 2];  // in 0..M: the plane holds the basis' weights
  for (int q = 0; q < 4; ++q)
    plane_lam[(b * 4 + q) * K2 + u2] = lam[(b * 4 + q) * K + u2 * (M + 1) + uk];
}

// 2-D spectrum of g(x, y, 0) from the stored 3-D octant: the inverse z
// transform at z = 0 is the sum over kz, i.e. over the folded kz with
// multiplicity 2 except kz = 0 and kz = Pz/2 (the normalisation carries over:
// octant / (Px Py Pz) summed over kz = 2-D spectrum / (Px Py))
__global__ void k_ghat_zsum(const double2 *oct, double2 *out, int Hx, int Hy, int Hz, int Pz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)Hx * Hy) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int z = 0; z < Hz; ++z) {
    const double m = (z == 0 || 2 * z == Pz) ? 1.0 : 2.0;
    const double2 v = oct[t * Hz + z];
    acc.x += m * v.x;
    acc.y += m * v.y;
  }
  out[t] = acc;
}

__global__ void k_extract_octant(const double2 *full, double2 *oct, int Py, int Pz, int Hx, int Hy,
                                 int Hz, double scale) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)Hx * Hy * Hz;
  if (t >= tot) return;
  const int kk = (int)(t % Hz);
  const int jj = (int)((t / Hz) % Hy);
  const int ii = (int)(t / ((int64_t)Hy * Hz));
  double2 v = full[((int64_t)ii * Py + jj) * Pz + kk];
  oct[t] = make_double2(v.x * scale, v.y * scale);
}

// g at integer offsets (i, j, k) in [0, D]^3 for the near-zone grid part
__global__ void k_green_table(double2 *tab, int D, double k, double h) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int D1 = D + 1;
  if (t >= D1 * D1 * D1) return;
  const int i = t / (D1 * D1), j = (t / D1) % D1, l = t % D1;
  tab[t] = green(k, h * sqrt((double)i * i + (double)j * j + (double)l * l));
}

// Z^near_mn = Z^MOM_mn - Z^grid_mn for the near pairs of row m = blockIdx.x
// (one thread per nonzero); diagonal Z^MOM_mm is also stored.
__global__ void __launch_bounds__(128)
    k_near_fill(const int32_t *rwg, const double *len, const double *area, const int32_t *tris,
                const double *verts, const int32_t *anchor3, const int32_t *rowptr,
                const int32_t *cols, const double *lam, const double *curl, double alpha,
                const double2 *gtab, int D, int M, double k, double eta, int64_t row0,
                double2 *nearv, double2 *zdiag) {
  extern __shared__ double lam_m[];  // 4 K projection weights, then 3 K curl weights (CFIE)
  const int K = (M + 1) * (M + 1) * (M + 1);
  const int64_t m = row0 + blockIdx.x;
  for (int i = threadIdx.x; i < 4 * K; i += blockDim.x) lam_m[i] = lam[m * 4 * K + i];
  double *w_m = lam_m + 4 * K;
  if (curl)
    for (int i = threadIdx.x; i < 3 * K; i += blockDim.x) w_m[i] = curl[m * 3 * K + i];
  __syncthreads();
  const double pref = k * eta;  // real factor of j k eta
  D3 Tm[2][3], pm[2];
  double Am[2], sm[2], lm = 0;
  int tm_id[2];
  for (int side = 0; side < 2; ++side) {
    basis_side(rwg, len, area, tris, verts, m, side, Tm[side], &Am[side], &pm[side], &sm[side], &lm);
    tm_id[side] = rwg[4 * m + side];
  }
  const int am[3] = {anchor3[3 * m], anchor3[3 * m + 1], anchor3[3 * m + 2]};
  const int D1 = D + 1;
  const int M1 = M + 1;
  for (int64_t e = rowptr[m] + threadIdx.x; e < rowptr[m + 1]; e += blockDim.x) {
    const int64_t n = cols[e];
    // ---- Z^MOM_mn from the four triangle pairs
    double zr = 0.0, zi = 0.0;
    for (int sn_ = 0; sn_ < 2; ++sn_) {
      D3 Tn[3], pn;
      double An, sn, ln;
      basis_side(rwg, len, area, tris, verts, n, sn_, Tn, &An, &pn, &sn, &ln);
      const int tn = rwg[4 * n + sn_];
      const int32_t *vn = &tris[3 * (int64_t)tn];
      for (int sm_ = 0; sm_ < 2; ++sm_) {
        const int32_t *vm = &tris[3 * (int64_t)tm_id[sm_]];
        bool touch = false;
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) touch |= (vm[a] == vn[c]);
        const C2 I = efie_pair(Tm[sm_], Am[sm_], pm[sm_], Tn, An, pn, k, touch);
        const double f = sm[sm_] * sn * lm * ln / (4.0 * Am[sm_] * An);
        zr += f * I.re;
        zi += f * I.im;
      }
    }
    // j k eta (zr + j zi)
    double mom_re = -pref * zi, mom_im = pref * zr;
    if (curl) {
      // combined field: alpha Z^E + (1 - alpha) eta (G/2 - K) over the four
      // triangle pairs (coplanar pairs, the same triangle included, have K = 0)
      double hr = 0.0, hi = 0.0;
      for (int sn_ = 0; sn_ < 2; ++sn_) {
        D3 Tn[3], pn;
        double An, sn, ln;
        basis_side(rwg, len, area, tris, verts, n, sn_, Tn, &An, &pn, &sn, &ln);
        const int tn = rwg[4 * n + sn_];
        const int32_t *vn = &tris[3 * (int64_t)tn];
        for (int sm_ = 0; sm_ < 2; ++sm_) {
          const double f = sm[sm_] * sn * lm * ln / (4.0 * Am[sm_] * An);
          if (tm_id[sm_] == tn) {
            hr += f * 0.5 * gram_pair(Tm[sm_], Am[sm_], pm[sm_], pn);
            continue;
          }
          if (coplanar(Tm[sm_], Tn)) continue;
          const int32_t *vm = &tris[3 * (int64_t)tm_id[sm_]];
          bool touch = false;
          for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) touch |= (vm[a] == vn[c]);
          const C2 I = mfie_pair(Tm[sm_], Am[sm_], pm[sm_], tri_normal(Tm[sm_]), Tn, An, pn, k, touch);
          hr -= f * I.re;
          hi -= f * I.im;
        }
      }
      mom_re = alpha * mom_re + (1.0 - alpha) * eta * hr;
      mom_im = alpha * mom_im + (1.0 - alpha) * eta * hi;
    }
    // ---- Z^grid_mn = j k eta [sum_{q<3} L_mq^T G L_nq - k^-2 L_md^T G L_nd]
    const int dn[3] = {am[0] - anchor3[3 * n], am[1] - anchor3[3 * n + 1], am[2] - anchor3[3 * n + 2]};
    const double *lam_n = lam + n * 4 * K;
    double gr = 0.0, gi = 0.0, wr = 0.0, wi = 0.0;
    for (int v = 0; v < K; ++v) {
      const int vi = v / (M1 * M1), vj = (v / M1) % M1, vk = v % M1;
      const double ln0 = lam_n[v], ln1 = lam_n[K + v], ln2 = lam_n[2 * K + v], ln3 = lam_n[3 * K + v];
      double tr0 = 0, ti0 = 0, tr1 = 0, ti1 = 0;  // vector and scalar parts
      double tr2 = 0, ti2 = 0;                    // curl-weight part (combined field)
      for (int u = 0; u < K; ++u) {
        const int ui = u / (M1 * M1), uj = (u / M1) % M1, uk = u % M1;
        const int oi = abs(dn[0] + ui - vi), oj = abs(dn[1] + uj - vj), ok = abs(dn[2] + uk - vk);
        const double2 g = gtab[(oi * D1 + oj) * D1 + ok];
        const double vec = lam_m[u] * ln0 + lam_m[K + u] * ln1 + lam_m[2 * K + u] * ln2;
        const double sca = lam_m[3 * K + u] * ln3;
        tr0 += g.x * vec;
        ti0 += g.y * vec;
        tr1 += g.x * sca;
        ti1 += g.y * sca;
        if (curl) {
          const double cw = w_m[u] * ln0 + w_m[K + u] * ln1 + w_m[2 * K + u] * ln2;
          tr2 += g.x * cw;
          ti2 += g.y * cw;
        }
      }
      gr += tr0 - tr1 / (k * k);
      gi += ti0 - ti1 / (k * k);
      wr += tr2;
      wi += ti2;
    }
    double grid_re = -pref * gi, grid_im = pref * gr;
    if (curl) {  // alpha j k eta [..] - (1 - alpha) eta W^T g Lambda
      grid_re = alpha * grid_re - (1.0 - alpha) * eta * wr;
      grid_im = alpha * grid_im - (1.0 - alpha) * eta * wi;
    }
    nearv[e] = make_double2(mom_re - grid_re, mom_im - grid_im);
    if (n == m) zdiag[m] = make_double2(mom_re, mom_im);
  }
}

__global__ void k_excitation(const int32_t *rwg, const double *len, const double *area,
                             const int32_t *tris, const double *verts, int64_t n, double k,
                             const double *wv /* per wave: khat(3), pol(3) */, int nw,
                             double alpha, bool cfie, double2 *b, int64_t ldb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nw) return;
  const int w = (int)(t / n);
  const int64_t m = t - (int64_t)w * n;
  const D3 kh = d3(wv[6 * w], wv[6 * w + 1], wv[6 * w + 2]);
  const D3 ph = d3(wv[6 * w + 3], wv[6 * w + 4], wv[6 * w + 5]);
  const D3 hd = cross(kh, ph);  // eta H_inc direction
  double vr = 0.0, vi = 0.0;
  for (int side = 0; side < 2; ++side) {
    D3 T[3], pf;
    double A, s, l;
    basis_side(rwg, len, area, tris, verts, m, side, T, &A, &pf, &s, &l);
    const double cf = s * l / (2.0 * A);
    // tested field direction: p_hat (EFIE); alpha p_hat + (1 - alpha) n x (k_hat x p_hat) (CFIE)
    const D3 dir = cfie ? alpha * ph + (1.0 - alpha) * cross(tri_normal(T), hd) : ph;
    for (int p = 0; p < 7; ++p) {
      double wq;
      const D3 r = quad_point(T, p, &wq);
      const double fp = cf * dot(r - pf, dir);
      double sn, cs;
      sincos(k * dot(kh, r), &sn, &cs);  // exp(-j k khat.r)
      vr += A * wq * fp * cs;
      vi -= A * wq * fp * sn;
    }
  }
  b[(int64_t)w * ldb + m] = make_double2(vr, vi);
}

int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

template <typename T>
static T *upload(Plan *pl, const T *host, size_t count, hipStream_t s) {
  T *d = (T *)dev_alloc(pl, count * sizeof(T));
  HIPCHECK(hipMemcpyAsync(d, host, count * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

static void twiddles(Plan *pl, int P, double2 **d64, float2 **d32, hipStream_t s) {
  std::vector<double2> w(P);
  std::vector<float2> wf(P);
  for (int e = 0; e < P; ++e) {
    long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)e / (long double)P;
    long double c = cosl(a), sn = sinl(a);
    w[e] = make_double2((double)c, (double)sn);
    wf[e] = make_float2((float)c, (float)sn);
  }
  *d64 = upload(pl, w.data(), P, s);
  *d32 = pl->mixed ? upload(pl, wf.data(), P, s) : nullptr;
  HIPCHECK(hipStreamSynchronize(s));  // host vectors go out of scope
}

void setup_mesh_device(Plan *pl, MeshDev &md, hipStream_t s) {
  const HostPlan &h = md.hp;
  const int M = h.order, K = h.K;
  const int64_t n = h.n;
  double t_phase = wall_ms();
  auto phase_done = [&](int which) {  // the stream is synchronised at each phase end
    const double t = wall_ms();
    md.setup_ms[which] = t - t_phase;
    t_phase = t;
  };
  // geometry and tables
  md.verts = upload(pl, h.verts.data(), h.verts.size(), s);
  md.tris = upload(pl, h.tris.data(), h.tris.size(), s);
  double *area = upload(pl, h.area.data(), h.area.size(), s);
  std::vector<int32_t> rwg(4 * n);
  std::vector<int32_t> alin(n);
  for (int64_t i = 0; i < n; ++i) {
    rwg[4 * i] = h.tp[i];
    rwg[4 * i + 1] = h.tm[i];
    rwg[4 * i + 2] = h.vp[i];
    rwg[4 * i + 3] = h.vm[i];
    alin[i] = (int32_t)(((int64_t)h.anchor[3 * i] * h.grid[1] + h.anchor[3 * i + 1]) * h.grid[2] +
                        h.anchor[3 * i + 2]);
  }
  md.rwg = upload(pl, rwg.data(), rwg.size(), s);
  md.len = upload(pl, h.len.data(), h.len.size(), s);
  md.anchor_lin = upload(pl, alin.data(), alin.size(), s);
  int32_t *anchor3 = upload(pl, h.anchor.data(), h.anchor.size(), s);
  std::vector<int32_t> soff(K);
  for (int u = 0; u < K; ++u) {
    int ui = u / ((M + 1) * (M + 1)), uj = (u / (M + 1)) % (M + 1), uk = u % (M + 1);
    soff[u] = (ui * h.grid[1] + uj) * h.grid[2] + uk;
  }
  md.stencil_off = upload(pl, soff.data(), soff.size(), s);
  std::vector<int32_t> rp32(n + 1);
  for (int64_t i = 0; i <= n; ++i) rp32[i] = (int32_t)h.rowptr[i];
  md.rowptr = upload(pl, rp32.data(), rp32.size(), s);
  md.cols = upload(pl, h.cols.data(), h.cols.size(), s);
  HIPCHECK(hipStreamSynchronize(s));

  // projection weights
  md.lam64 = (double *)dev_alloc(pl, sizeof(double) * n * 4 * K);
  hipLaunchKernelGGL(k_projection, dim3(blocks_for(n * K, 256)), dim3(256), 0, s, md.rwg, md.len,
                     area, md.tris, md.verts, anchor3, n, M, h.x0[0], h.x0[1], h.x0[2], h.h,
                     md.lam64);
  LAUNCHCHECK();
  if (pl->mixed) {
    md.lam32 = (float *)dev_alloc(pl, sizeof(float) * n * 4 * K);
    hipLaunchKernelGGL(k_to_float, dim3(blocks_for(n * 4 * K, 256)), dim3(256), 0, s, md.lam64,
                       md.lam32, n * 4 * K);
    LAUNCHCHECK();
  }
  if (h.cfie) {  // curl weights of the MFIE part
    md.curl64 = (double *)dev_alloc(pl, sizeof(double) * n * 3 * K);
    hipLaunchKernelGGL(k_curl_projection, dim3(blocks_for(n * K, 256)), dim3(256), 0, s, md.rwg,
                       md.len, area, md.tris, md.verts, anchor3, n, M, h.x0[0], h.x0[1], h.x0[2],
                       h.h, md.curl64);
    LAUNCHCHECK();
    if (pl->mixed) {
      md.curl32 = (float *)dev_alloc(pl, sizeof(float) * n * 3 * K);
      hipLaunchKernelGGL(k_to_float, dim3(blocks_for(n * 3 * K, 256)), dim3(256), 0, s, md.curl64,
                         md.curl32, n * 3 * K);
      LAUNCHCHECK();
    }
  }

  // a flat scatterer lying in one grid plane: every projection weight on
  // that plane (exactly: the off-plane Lagrange factors vanish), so the
  // propagation and the interpolation reduce to the plane
  {
    int zr_h[2] = {INT32_MAX, INT32_MIN};
    int *zr = upload(pl, zr_h, 2, s);
    hipLaunchKernelGGL(k_lam_zrange, dim3(blocks_for(n * K, 256)), dim3(256), 0, s, md.lam64,
                       anchor3, n, M, zr);
    LAUNCHCHECK();
    HIPCHECK(hipMemcpyAsync(zr_h, zr, sizeof(zr_h), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    dev_free(pl, zr);
    md.planar_z = (n > 0 && zr_h[0] == zr_h[1]) ? zr_h[0] : -1;
  }
  if (md.planar_z >= 0) {
    // in-plane stencils: (M+1)^2 weights per component, plane-linear anchors
    const int K2 = (M + 1) * (M + 1);
    md.plane_lam64 = (double *)dev_alloc(pl, sizeof(double) * n * 4 * K2);
    hipLaunchKernelGGL(k_lam_plane, dim3(blocks_for(n * K2, 256)), dim3(256), 0, s, md.lam64,
                       anchor3, n, M, md.planar_z, md.plane_lam64);
    LAUNCHCHECK();
    if (pl->mixed) {
      md.plane_lam32 = (float *)dev_alloc(pl, sizeof(float) * n * 4 * K2);
      hipLaunchKernelGGL(k_to_float, dim3(blocks_for(n * 4 * K2, 256)), dim3(256), 0, s,
                         md.plane_lam64, md.plane_lam32, n * 4 * K2);
      LAUNCHCHECK();
    }
    std::vector<int32_t> a2(n), so2(K2);
    for (int64_t i = 0; i < n; ++i) a2[i] = h.anchor[3 * i] * h.grid[1] + h.anchor[3 * i + 1];
    for (int u = 0; u < K2; ++u) so2[u] = (u / (M + 1)) * h.grid[1] + u % (M + 1);
    md.plane_anchor = upload(pl, a2.data(), a2.size(), s);
    md.plane_soff = upload(pl, so2.data(), so2.size(), s);
    md.plane_K = K2;
  }

  // node-ordered (transposed) projection for the gather form of anterpolation
  {
    const int64_t NK = n * K;
    uint8_t *dmask = (uint8_t *)dev_alloc(pl, NK);
    hipLaunchKernelGGL(k_lam_mask, dim3(blocks_for(NK, 256)), dim3(256), 0, s, md.lam64, md.curl64,
                       n, K, dmask);
    LAUNCHCHECK();
    std::vector<uint8_t> mask(NK);
    HIPCHECK(hipMemcpyAsync(mask.data(), dmask, NK, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    dev_free(pl, dmask);
    const int64_t V0 = (int64_t)h.grid[0] * h.grid[1] * h.grid[2];
    std::vector<int32_t> ptr(V0 + 1, 0);
    for (int64_t b = 0; b < n; ++b)
      for (int u = 0; u < K; ++u)
        if (mask[b * K + u]) ptr[alin[b] + soff[u] + 1]++;
    for (int64_t v = 0; v < V0; ++v) ptr[v + 1] += ptr[v];
    const int64_t ne = ptr[V0];
    if (ne > INT32_MAX) throw Error(AIM_ERR_ARG, "projection too large for 32-bit indexing");
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1), col(std::max<int64_t>(ne, 1)),
        src(std::max<int64_t>(ne, 1));
    for (int64_t b = 0; b < n; ++b)  // entries of a node in (basis, node) order
      for (int u = 0; u < K; ++u)
        if (mask[b * K + u]) {
          const int32_t e = fill[alin[b] + soff[u]]++;
          col[e] = (int32_t)b;
          src[e] = (int32_t)(b * K + u);
        }
    md.n_entries = ne;
    md.node_ptr = upload(pl, ptr.data(), ptr.size(), s);
    {
      std::vector<int32_t> occ, optr;
      for (int64_t v = 0; v < V0; ++v)
        if (ptr[v + 1] > ptr[v]) {
          occ.push_back((int32_t)v);
          optr.push_back(ptr[v]);
        }
      optr.push_back(ptr[V0]);
      std::vector<int32_t> lines;
      for (int32_t v : occ)
        if (lines.empty() || lines.back() != v / h.grid[2]) lines.push_back(v / h.grid[2]);
      md.n_occ = (int64_t)occ.size();
      md.n_occ_lines = (int64_t)lines.size();
      if (occ.empty()) occ.push_back(0);
      if (lines.empty()) lines.push_back(0);
      md.occ = upload(pl, occ.data(), occ.size(), s);
      md.occ_ptr = upload(pl, optr.data(), optr.size(), s);
      md.occ_lines = upload(pl, lines.data(), lines.size(), s);
      std::vector<int32_t> yr(2 * (size_t)h.grid[0], 0);
      for (int64_t x = 0; x < h.grid[0]; ++x) yr[2 * x] = h.grid[1];
      for (int64_t i = 0; i < md.n_occ_lines; ++i) {
        const int64_t x = lines[i] / h.grid[1], y = lines[i] % h.grid[1];
        yr[2 * x] = std::min<int32_t>(yr[2 * x], (int32_t)y);
        yr[2 * x + 1] = std::max<int32_t>(yr[2 * x + 1], (int32_t)y + 1);
      }
      for (int64_t x = 0; x < h.grid[0]; ++x)
        if (yr[2 * x] > yr[2 * x + 1]) yr[2 * x] = yr[2 * x + 1] = 0;
      md.occ_yrange = upload(pl, yr.data(), yr.size(), s);
      // per occupied line {lo, g0, g1, hi}: its occupied nodes lie in
      // [lo, hi) outside the longest unoccupied run [g0, g1) between them (a
      // line through a closed surface crosses it twice); occupied nodes are
      // increasing, so lines come in order
      std::vector<int32_t> zr;
      for (int64_t i = 0; i < md.n_occ; ++i) {
        const int32_t line = occ[i] / h.grid[2], z = occ[i] % h.grid[2];
        if (zr.empty() || line != occ[i - 1] / h.grid[2]) {
          zr.insert(zr.end(), {z, z + 1, z + 1, z + 1});
        } else {
          int32_t *r = &zr[zr.size() - 4];
          if (z - r[3] > r[2] - r[1]) {  // a longer unoccupied run r[3] .. z - 1
            r[1] = r[3];
            r[2] = z;
          }
          r[3] = z + 1;
        }
      }
      if (zr.empty()) zr.assign(4, 0);
      md.occ_zrange = upload(pl, zr.data(), zr.size(), s);
      HIPCHECK(hipStreamSynchronize(s));  // host vectors go out of scope
    }
    if (md.planar_z >= 0) {  // all entries sit on the plane: plane node p = x Ny + y
      const int64_t A = (int64_t)h.grid[0] * h.grid[1];
      std::vector<int32_t> p2(A + 1);
      for (int64_t p = 0; p < A; ++p) p2[p] = ptr[p * h.grid[2] + md.planar_z];
      p2[A] = ptr[V0];
      md.plane_node_ptr = upload(pl, p2.data(), p2.size(), s);
      std::vector<int32_t> occ, optr;
      for (int64_t p = 0; p < A; ++p)
        if (p2[p + 1] > p2[p]) {
          occ.push_back((int32_t)p);
          optr.push_back(p2[p]);
        }
      optr.push_back(p2[A]);
      md.n_plane_occ = (int64_t)occ.size();
      if (occ.empty()) occ.push_back(0);
      md.plane_occ = upload(pl, occ.data(), occ.size(), s);
      md.plane_occ_ptr = upload(pl, optr.data(), optr.size(), s);
      HIPCHECK(hipStreamSynchronize(s));  // host vectors go out of scope
    }
    md.ent_col = upload(pl, col.data(), col.size(), s);
    int32_t *dsrc = upload(pl, src.data(), src.size(), s);
    md.lamT64 = (double *)dev_alloc(pl, sizeof(double) * 4 * std::max<int64_t>(ne, 1));
    if (pl->mixed) md.lamT32 = (float *)dev_alloc(pl, sizeof(float) * 4 * std::max<int64_t>(ne, 1));
    hipLaunchKernelGGL(k_lam_transpose, dim3(blocks_for(std::max<int64_t>(ne, 1), 256)), dim3(256), 0,
                       s, md.lam64, dsrc, ne, K, md.lamT64, md.lamT32);
    LAUNCHCHECK();
    HIPCHECK(hipStreamSynchronize(s));
    dev_free(pl, dsrc);
  }
  phase_done(AIM_SETUP_PROJECTION);

  // FFT plans, twiddles, Green's spectrum octant
  for (int d = 0; d < 3; ++d) {
    if (!fft_plan_for(h.pad[d], &md.plan[d])) throw Error(AIM_ERR_ARG, "unsupported FFT length");
    md.H[d] = h.pad[d] / 2 + 1;
    twiddles(pl, h.pad[d], &md.tw64[d], &md.tw32[d], s);
  }
  {
    const int Px = h.pad[0], Py = h.pad[1], Pz = h.pad[2];
    const int64_t tot = (int64_t)Px * Py * Pz;
    double2 *e0 = (double2 *)dev_alloc(pl, sizeof(double2) * tot);
    double2 *e1 = (double2 *)dev_alloc(pl, sizeof(double2) * tot);
    hipLaunchKernelGGL(k_embed_green, dim3(blocks_for(tot, 256)), dim3(256), 0, s, e0, Px, Py, Pz,
                       h.grid[0], h.grid[1], h.grid[2], h.k, h.h);
    LAUNCHCHECK();
    fft_pass_contig(e0, e1, md.plan[2], Pz, Pz, (int64_t)Px * Py, fftk::contig_map(Pz),
                    fftk::contig_map(Pz), false, md.tw64[2], s);
    const fftk::LineMap my = fftk::plain_map((int64_t)Py * Pz, Pz);
    const fftk::LineMap mx = fftk::plain_map(0, (int64_t)Py * Pz);
    fft_pass_strided(e1, e0, md.plan[1], Py, Py, Px, Pz, my, my, false, md.tw64[1], 128, s);
    fft_pass_strided(e0, e1, md.plan[0], Px, Px, 1, (int64_t)Py * Pz, mx, mx, false, md.tw64[0],
                     128, s);
    const int64_t noct = (int64_t)md.H[0] * md.H[1] * md.H[2];
    md.ghat64 = (double2 *)dev_alloc(pl, sizeof(double2) * noct);
    hipLaunchKernelGGL(k_extract_octant, dim3(blocks_for(noct, 256)), dim3(256), 0, s, e1,
                       md.ghat64, Py, Pz, md.H[0], md.H[1], md.H[2], 1.0 / (double)tot);
    LAUNCHCHECK();
    if (pl->mixed) {
      md.ghat32 = (float2 *)dev_alloc(pl, sizeof(float2) * noct);
      hipLaunchKernelGGL(k_to_float, dim3(blocks_for(2 * noct, 256)), dim3(256), 0, s,
                         (const double *)md.ghat64, (float *)md.ghat32, 2 * noct);
      LAUNCHCHECK();
    }
    HIPCHECK(hipStreamSynchronize(s));
    dev_free(pl, e0);
    dev_free(pl, e1);
  }
  if (md.planar_z >= 0) {
    const int64_t n2 = (int64_t)md.H[0] * md.H[1];
    md.ghat2d64 = (double2 *)dev_alloc(pl, sizeof(double2) * n2);
    hipLaunchKernelGGL(k_ghat_zsum, dim3(blocks_for(n2, 256)), dim3(256), 0, s, md.ghat64,
                       md.ghat2d64, md.H[0], md.H[1], md.H[2], h.pad[2]);
    LAUNCHCHECK();
    if (pl->mixed) {
      md.ghat2d32 = (float2 *)dev_alloc(pl, sizeof(float2) * n2);
      hipLaunchKernelGGL(k_to_float, dim3(blocks_for(2 * n2, 256)), dim3(256), 0, s,
                         (const double *)md.ghat2d64, (float *)md.ghat2d32, 2 * n2);
      LAUNCHCHECK();
    }
    HIPCHECK(hipStreamSynchronize(s));
  }
  phase_done(AIM_SETUP_GREEN);

  // near zone: offsets table size from the largest anchor difference
  int D = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = h.rowptr[i]; e < h.rowptr[i + 1]; ++e) {
      const int64_t j = h.cols[e];
      for (int c = 0; c < 3; ++c) D = std::max(D, std::abs(h.anchor[3 * i + c] - h.anchor[3 * j + c]));
    }
  D += M;
  const int D1 = D + 1;
  double2 *gtab = (double2 *)dev_alloc(pl, sizeof(double2) * D1 * D1 * D1);
  hipLaunchKernelGGL(k_green_table, dim3(blocks_for((int64_t)D1 * D1 * D1, 256)), dim3(256), 0, s,
                     gtab, D, h.k, h.h);
  LAUNCHCHECK();
  md.near64 = (double2 *)dev_alloc(pl, sizeof(double2) * std::max<int64_t>(h.nnz, 1));
  md.zdiag = (double2 *)dev_alloc(pl, sizeof(double2) * n);
  const int64_t chunk = 1 << 20;  // rows per launch
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int64_t rows = std::min(chunk, n - r0);
    hipLaunchKernelGGL(k_near_fill, dim3((unsigned)rows), dim3(128),
                       sizeof(double) * (h.cfie ? 7 : 4) * K, s, md.rwg, md.len, area, md.tris,
                       md.verts, anchor3, md.rowptr, md.cols, md.lam64, md.curl64, h.alpha, gtab,
                       D, M, h.k, kEta0, r0, md.near64, md.zdiag);
    LAUNCHCHECK();
  }
  if (pl->mixed) {
    md.near32 = (float2 *)dev_alloc(pl, sizeof(float2) * std::max<int64_t>(h.nnz, 1));
    hipLaunchKernelGGL(k_to_float, dim3(blocks_for(2 * h.nnz, 256)), dim3(256), 0, s,
                       (const double *)md.near64, (float *)md.near32, 2 * h.nnz);
    LAUNCHCHECK();
  }
  HIPCHECK(hipStreamSynchronize(s));
  phase_done(AIM_SETUP_NEAR_FILL);
  dev_free(pl, gtab);
  dev_free(pl, anchor3);
  md.area = area;  // kept for excitation and RCS
  rcs_prepare_mesh(pl, md, s);
}

void excitation_mesh(Plan *pl, MeshDev &md, int nw, const aim_planewave *w, double2 *b,
                     int64_t ldb, hipStream_t s) {
  (void)pl;
  std::vector<double> wv(6 * nw);
  for (int i = 0; i < nw; ++i) {
    const double st = std::sin(w[i].theta), ct = std::cos(w[i].theta);
    const double sp = std::sin(w[i].phi), cp = std::cos(w[i].phi);
    // k_hat = -r_hat; p_hat = theta_hat or phi_hat
    wv[6 * i + 0] = -st * cp;
    wv[6 * i + 1] = -st * sp;
    wv[6 * i + 2] = -ct;
    if (w[i].pol == 0) {
      wv[6 * i + 3] = ct * cp;
      wv[6 * i + 4] = ct * sp;
      wv[6 * i + 5] = -st;
    } else {
      wv[6 * i + 3] = -sp;
      wv[6 * i + 4] = cp;
      wv[6 * i + 5] = 0.0;
    }
  }
  double *dwv = upload(pl, wv.data(), wv.size(), s);
  const int64_t n = md.hp.n;
  hipLaunchKernelGGL(k_excitation, dim3(blocks_for(n * nw, 256)), dim3(256), 0, s, md.rwg, md.len,
                     md.area, md.tris, md.verts, n, md.hp.k, dwv, nw, md.hp.alpha, md.hp.cfie, b,
                     ldb);
  LAUNCHCHECK();
  HIPCHECK(hipStreamSynchronize(s));
  dev_free(pl, dwv);
}

}  // namespace aim
