// Device-side geometry helpers: the 7-point triangle rule, RWG evaluation,
// closed-form static potentials of a triangle, and the EFIE triangle-pair
// integral in FP64 (used by the set-up kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace aim {
namespace geo {

// Radon's 7-point rule (degree 5): barycentric points and weights (sum 1).
// a = (6 - sqrt 15)/21, b = (6 + sqrt 15)/21, w_a = (155 - sqrt 15)/1200,
// w_b = (155 + sqrt 15)/1200, centre weight 9/40.
constexpr double kQa = 0.10128650732345633880098736191512;
constexpr double kQb = 0.47014206410511508977044120951345;
constexpr double kWa = 0.12593918054482715259568394550018;
constexpr double kWb = 0.13239415278850618073764938783315;
constexpr double kWc = 0.225;

__host__ __device__ inline void quad_bary(int p, double &l0, double &l1, double &l2, double &w) {
  const double c = 1.0 / 3.0;
  switch (p) {
    case 0: l0 = c; l1 = c; l2 = c; w = kWc; break;
    case 1: l0 = 1.0 - 2.0 * kQa; l1 = kQa; l2 = kQa; w = kWa; break;
    case 2: l0 = kQa; l1 = 1.0 - 2.0 * kQa; l2 = kQa; w = kWa; break;
    case 3: l0 = kQa; l1 = kQa; l2 = 1.0 - 2.0 * kQa; w = kWa; break;
    case 4: l0 = 1.0 - 2.0 * kQb; l1 = kQb; l2 = kQb; w = kWb; break;
    case 5: l0 = kQb; l1 = 1.0 - 2.0 * kQb; l2 = kQb; w = kWb; break;
    default: l0 = kQb; l1 = kQb; l2 = 1.0 - 2.0 * kQb; w = kWb; break;
  }
}

struct D3 {
  double x, y, z;
};
__host__ __device__ inline D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__host__ __device__ inline D3 operator+(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline D3 operator-(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline D3 operator*(double s, D3 a) { return d3(s * a.x, s * a.y, s * a.z); }
__host__ __device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline D3 cross(D3 a, D3 b) {
  return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double norm(D3 a) { return sqrt(dot(a, a)); }

__host__ __device__ inline D3 vtx(const double *verts, int v) {
  return d3(verts[3 * (int64_t)v], verts[3 * (int64_t)v + 1], verts[3 * (int64_t)v + 2]);
}

__host__ __device__ inline D3 quad_point(const D3 *T, int p, double *w) {
  double l0, l1, l2;
  quad_bary(p, l0, l1, l2, *w);
  return l0 * T[0] + l1 * T[1] + l2 * T[2];
}

// R + l computed without cancellation (R^2 = l^2 + R0^2)
__host__ __device__ inline double r_plus_l(double R, double l, double R0sq) {
  return l >= 0.0 ? R + l : R0sq / (R - l);
}

// I1 = int_T 1/|r - r'| dS', Iv = int_T (r' - r)/|r - r'| dS' (Wilton et al.
// 1984; Graglia 1993), for a planar triangle T and observation point r.
__host__ __device__ inline void triangle_potentials(const D3 *T, D3 r, double &I1, D3 &Iv) {
  D3 n = cross(T[1] - T[0], T[2] - T[0]);
  n = (1.0 / norm(n)) * n;
  const double d = dot(r - T[0], n);
  const double ad = fabs(d);
  const D3 rho = r - d * n;
  double acc1 = 0.0;
  D3 accv = d3(0, 0, 0);
  for (int e = 0; e < 3; ++e) {
    const D3 a = T[e], b = T[(e + 1) % 3];
    D3 lhat = b - a;
    lhat = (1.0 / norm(lhat)) * lhat;
    const D3 uhat = cross(lhat, n);
    const double t0 = dot(a - rho, uhat);
    const double lp = dot(b - rho, lhat);
    const double lm = dot(a - rho, lhat);
    const double R0sq = t0 * t0 + d * d;
    const double Rp = sqrt(lp * lp + R0sq);
    const double Rm = sqrt(lm * lm + R0sq);
    double f = 0.0, atp = 0.0, atm = 0.0;
    if (R0sq > 0.0) {
      f = log(r_plus_l(Rp, lp, R0sq)) - log(r_plus_l(Rm, lm, R0sq));
      atp = atan2(t0 * lp, R0sq + ad * Rp);
      atm = atan2(t0 * lm, R0sq + ad * Rm);
    }
    acc1 += t0 * f - ad * (atp - atm);
    accv = accv + (0.5 * (R0sq * f + lp * Rp - lm * Rm)) * uhat;
  }
  I1 = acc1;
  Iv = accv - (d * acc1) * n;
}

// G1 = int_T grad_r 1/|r - r'| dS' and Iv (as above) for a planar triangle.
// In-plane part of G1 by the divergence theorem (minus the edge integrals of
// 1/R along the outward edge normals: - sum_i u_i f_i); normal part the
// d-derivative of I1, -sign(d) times the solid angle of T seen from r (the
// arctan sum), zero in the plane of T.
__host__ __device__ inline void triangle_gradient(const D3 *T, D3 r, D3 &G1, D3 &Iv) {
  D3 n = cross(T[1] - T[0], T[2] - T[0]);
  n = (1.0 / norm(n)) * n;
  const double d = dot(r - T[0], n);
  const double ad = fabs(d);
  const D3 rho = r - d * n;
  double acc1 = 0.0, omega = 0.0;
  D3 accv = d3(0, 0, 0), accg = d3(0, 0, 0);
  for (int e = 0; e < 3; ++e) {
    const D3 a = T[e], b = T[(e + 1) % 3];
    D3 lhat = b - a;
    lhat = (1.0 / norm(lhat)) * lhat;
    const D3 uhat = cross(lhat, n);
    const double t0 = dot(a - rho, uhat);
    const double lp = dot(b - rho, lhat);
    const double lm = dot(a - rho, lhat);
    const double R0sq = t0 * t0 + d * d;
    const double Rp = sqrt(lp * lp + R0sq);
    const double Rm = sqrt(lm * lm + R0sq);
    double f = 0.0, atp = 0.0, atm = 0.0;
    if (R0sq > 0.0) {
      f = log(r_plus_l(Rp, lp, R0sq)) - log(r_plus_l(Rm, lm, R0sq));
      atp = atan2(t0 * lp, R0sq + ad * Rp);
      atm = atan2(t0 * lm, R0sq + ad * Rm);
    }
    acc1 += t0 * f - ad * (atp - atm);
    omega += atp - atm;
    accv = accv + (0.5 * (R0sq * f + lp * Rp - lm * Rm)) * uhat;
    accg = accg - f * uhat;
  }
  const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
  G1 = accg - (sg * omega) * n;
  Iv = accv - (d * acc1) * n;
}

struct C2 {
  double re, im;
};

// true if every vertex of Tn lies in the plane of Tm (relative tolerance
// 1e-12 of the longer first edge): then the MFIE pair term vanishes
__host__ __device__ inline bool coplanar(const D3 *Tm, const D3 *Tn) {
  D3 n = cross(Tm[1] - Tm[0], Tm[2] - Tm[0]);
  n = (1.0 / norm(n)) * n;
  const double sc = fmax(norm(Tm[1] - Tm[0]), norm(Tn[1] - Tn[0]));
  for (int v = 0; v < 3; ++v)
    if (fabs(dot(Tn[v] - Tm[0], n)) > 1e-12 * sc) return false;
  return true;
}

// K pair factor of the MFIE for test triangle Tm (free vertex pm, outward
// normal nm) and a non-coplanar source triangle Tn (free vertex pn):
//   int_Tm [(r - pm) x nm] . [J(r) x (r - pn)] dS,  J(r) = int_Tn grad_r G dS'
// (grad G is parallel to r - r', so the source factor r' - pn becomes r - pn).
// The RWG pair contribution is s_m s_n l_m l_n / (4 A_m A_n) times this.
// `touch`: the first two terms of grad G in powers of R are integrated in
// closed form, -(r - r')/(4 pi R^3) (G1) and -k^2 (r - r')/(8 pi R) (Iv), and
// the smooth remainder (d/R) k^2/(4 pi) phi(kR) by the 7-point rule, with
// phi(x) = (1 - (1 + j x) exp(-j x))/x^2 + 1/2 (series below x = 1e-2).
__host__ __device__ inline C2 mfie_pair(const D3 *Tm, double Am, D3 pm, D3 nm, const D3 *Tn,
                                        double An, D3 pn, double k, bool touch) {
  const double inv4pi = 0.25 / 3.14159265358979323846;
  double sre = 0.0, sim = 0.0;
  for (int p = 0; p < 7; ++p) {
    double wp;
    const D3 rp = quad_point(Tm, p, &wp);
    D3 jr = d3(0, 0, 0), ji = d3(0, 0, 0);
    if (touch) {
      D3 G1, Iv;
      triangle_gradient(Tn, rp, G1, Iv);
      jr = inv4pi * G1 + (0.5 * k * k * inv4pi) * Iv;
    }
    for (int q = 0; q < 7; ++q) {
      double wq;
      const D3 rq = quad_point(Tn, q, &wq);
      const D3 dv = rp - rq;
      const double R = norm(dv);
      if (R == 0.0) continue;
      double gr, gi;  // radial factor: grad = (gr + j gi) dv
      if (!touch) {
        // grad G = -(1 + j k R) exp(-j k R) / (4 pi R^3) dv
        double sn, cs;
        sincos(k * R, &sn, &cs);
        const double c = -inv4pi / (R * R * R);
        gr = c * (cs + k * R * sn);
        gi = c * (k * R * cs - sn);
      } else {
        const double x = k * R;
        double pr, pi;
        if (x < 1e-2) {
          const double x2 = x * x;
          pr = x2 / 8.0 - x2 * x2 / 144.0;
          pi = x / 3.0 - x2 * x / 30.0;
        } else {
          double sn, cs;
          sincos(x, &sn, &cs);
          // (1 + j x)(cos x - j sin x) = (cos x + x sin x) + j (x cos x - sin x)
          pr = (1.0 - (cs + x * sn)) / (x * x) + 0.5;
          pi = -(x * cs - sn) / (x * x);
        }
        const double c = k * k * inv4pi / R;
        gr = c * pr;
        gi = c * pi;
      }
      const double a = An * wq;
      jr = jr + (a * gr) * dv;
      ji = ji + (a * gi) * dv;
    }
    // [(r - pm) x nm] . [J x (r - pn)] = J . [(r - pn) x ((r - pm) x nm)]
    const D3 cvec = cross(rp - pn, cross(rp - pm, nm));
    sre += wp * dot(jr, cvec);
    sim += wp * dot(ji, cvec);
  }
  return C2{sre * Am, sim * Am};
}

// int_T (r - pm) . (r - pn) dS by the 7-point rule (exact: quadratic)
__host__ __device__ inline double gram_pair(const D3 *T, double A, D3 pm, D3 pn) {
  double s = 0.0;
  for (int p = 0; p < 7; ++p) {
    double wp;
    const D3 rp = quad_point(T, p, &wp);
    s += wp * dot(rp - pm, rp - pn);
  }
  return s * A;
}

// Integral over test triangle Tm (free vertex pm) and source triangle Tn (free
// vertex pn) of [(r - pm).(r' - pn) - 4/k^2] G(|r - r'|), i.e. the factor I of
// the RWG pair contribution j k eta s_m s_n l_m l_n / (4 A_m A_n) * I.
// `touch`: the triangles share a vertex, so the inner integral is split into
// the closed-form static part and a 7-point rule of (exp(-jkR) - 1)/R.
__host__ __device__ inline C2 efie_pair(const D3 *Tm, double Am, D3 pm, const D3 *Tn, double An,
                                        D3 pn, double k, bool touch) {
  const double inv4pi = 0.25 / 3.14159265358979323846;
  const double c4k2 = 4.0 / (k * k);
  double sre = 0.0, sim = 0.0;
  if (!touch) {
    for (int p = 0; p < 7; ++p) {
      double wp;
      const D3 rp = quad_point(Tm, p, &wp);
      const D3 ap = rp - pm;
      for (int q = 0; q < 7; ++q) {
        double wq;
        const D3 rq = quad_point(Tn, q, &wq);
        const double R = norm(rp - rq);
        double sn, cs;
        sincos(k * R, &sn, &cs);
        const double g = inv4pi / R;  // G = (cos kR - j sin kR) / (4 pi R)
        const double br = dot(ap, rq - pn) - c4k2;
        const double ww = wp * wq * br * g;
        sre += ww * cs;
        sim -= ww * sn;
      }
    }
    return C2{sre * Am * An, sim * Am * An};
  }
  for (int p = 0; p < 7; ++p) {
    double wp;
    const D3 rp = quad_point(Tm, p, &wp);
    double I1;
    D3 Iv;
    triangle_potentials(Tn, rp, I1, Iv);
    // J1 = int G, Jr = int (r' - r) G over Tn
    double j1r = I1 * inv4pi, j1i = 0.0;
    D3 jrr = inv4pi * Iv, jri = d3(0, 0, 0);
    for (int q = 0; q < 7; ++q) {
      double wq;
      const D3 rq = quad_point(Tn, q, &wq);
      const D3 dv = rq - rp;
      const double R = norm(dv);
      double er, ei;  // (exp(-jkR) - 1) / R
      if (R == 0.0) {
        er = 0.0;
        ei = -k;
      } else {
        double sn, cs;
        sincos(k * R, &sn, &cs);
        er = (cs - 1.0) / R;
        ei = -sn / R;
      }
      const double a = An * wq * inv4pi;
      j1r += a * er;
      j1i += a * ei;
      jrr = jrr + (a * er) * dv;
      jri = jri + (a * ei) * dv;
    }
    const D3 ap = rp - pm;
    const D3 bp = rp - pn;
    // ap . (Jr + bp J1) - 4/k^2 J1
    const double vr = dot(ap, jrr) + dot(ap, bp) * j1r - c4k2 * j1r;
    const double vi = dot(ap, jri) + dot(ap, bp) * j1i - c4k2 * j1i;
    sre += wp * vr;
    sim += wp * vi;
  }
  return C2{sre * Am, sim * Am};
}

}  // namespace geo
}  // namespace aim
