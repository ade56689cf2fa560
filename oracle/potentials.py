"""Closed-form static potential integrals over a planar triangle.

Test infrastructure only. Singularity extraction on self and adjacent
triangle pairs needs, at an observation point r,

    I1(r)  = integral over T' of 1 / |r - r'| dS'
    Iv(r)  = integral over T' of (r' - r) / |r - r'| dS'

in closed form (Wilton, Rao, Glisson, Schaubert, Al-Bundak, Butler, IEEE
TAP 1984; Graglia, IEEE TAP 1993). With n the unit normal of T', d the
signed height of r above the plane, rho the projection of r, and for each
edge i with unit tangent l_i (counter-clockwise about n) and outward in-plane
normal u_i = l_i x n:

    t_i = (a_i - rho) . u_i,  l_i^-+ = (end points - rho) . l_i,
    R0_i^2 = t_i^2 + d^2,     R_i^-+ = sqrt(l_i^-+^2 + R0_i^2),
    f_i = ln((R_i^+ + l_i^+) / (R_i^- + l_i^-))

    I1 = sum_i [ t_i f_i - |d| ( atan(t_i l_i^+ / (R0_i^2 + |d| R_i^+))
                                - atan(t_i l_i^- / (R0_i^2 + |d| R_i^-)) ) ]
    integral of (rho' - rho)/R = 1/2 sum_i u_i [ R0_i^2 f_i + l_i^+ R_i^+ - l_i^- R_i^- ]
    Iv = that - d n I1

R + l is evaluated as R0^2 / (R - l) when l < 0 to avoid cancellation; when
R0 = 0 (r on the line of an edge) the edge's log term has limit zero.
"""

from __future__ import annotations

import numpy as np


def _log_ratio(Rp, lp, Rm, lm, R0sq):
    def rpl(R, l):
        out = np.empty_like(R)
        pos = l >= 0
        out[pos] = R[pos] + l[pos]
        neg = ~pos
        out[neg] = R0sq[neg] / (R[neg] - l[neg])
        return out

    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.log(rpl(Rp, lp)) - np.log(rpl(Rm, lm))
    return np.where(R0sq > 0.0, f, 0.0)


def triangle_potentials(tri: np.ndarray, r: np.ndarray):
    """I1 (P,) and Iv (P,3) for triangle ``tri`` (3,3) at points ``r`` (P,3)."""
    tri = np.asarray(tri, dtype=np.float64)
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    v0, v1, v2 = tri
    n = np.cross(v1 - v0, v2 - v0)
    n = n / np.linalg.norm(n)
    d = (r - v0) @ n
    rho = r - d[:, None] * n
    ad = np.abs(d)
    I1 = np.zeros(r.shape[0])
    Ip = np.zeros((r.shape[0], 3))
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        lhat = (b - a) / np.linalg.norm(b - a)
        uhat = np.cross(lhat, n)
        t0 = (a - rho) @ uhat
        lp = (b - rho) @ lhat
        lm = (a - rho) @ lhat
        R0sq = t0 * t0 + d * d
        Rp = np.sqrt(lp * lp + R0sq)
        Rm = np.sqrt(lm * lm + R0sq)
        f = _log_ratio(Rp, lp, Rm, lm, R0sq)
        with np.errstate(divide="ignore", invalid="ignore"):
            atp = np.where(R0sq > 0.0, np.arctan2(t0 * lp, R0sq + ad * Rp), 0.0)
            atm = np.where(R0sq > 0.0, np.arctan2(t0 * lm, R0sq + ad * Rm), 0.0)
        I1 += t0 * f - ad * (atp - atm)
        Ip += 0.5 * np.outer(R0sq * f + lp * Rp - lm * Rm, uhat)
    Iv = Ip - (d * I1)[:, None] * n
    return I1, Iv


def triangle_gradient(tri: np.ndarray, r: np.ndarray) -> np.ndarray:
    """G1(r) = integral over T' of grad_r 1/|r - r'| dS', (P, 3), in closed form.

    The in-plane part follows from the divergence theorem on T' (the gradient
    moves onto r' with a sign change and becomes a boundary integral of 1/R
    along each edge, which is the edge's log term f_i); the normal part is the
    d-derivative of I1, -sign(d) times the solid angle Omega that T' subtends
    at r (Omega is the bracketed arctan sum of I1):

        G1 = - sum_i u_i f_i - n sign(d) Omega.

    At d = 0 the normal part is taken as zero (its principal value)."""
    tri = np.asarray(tri, dtype=np.float64)
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    v0, v1, v2 = tri
    n = np.cross(v1 - v0, v2 - v0)
    n = n / np.linalg.norm(n)
    d = (r - v0) @ n
    rho = r - d[:, None] * n
    ad = np.abs(d)
    omega = np.zeros(r.shape[0])
    g = np.zeros((r.shape[0], 3))
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        lhat = (b - a) / np.linalg.norm(b - a)
        uhat = np.cross(lhat, n)
        t0 = (a - rho) @ uhat
        lp = (b - rho) @ lhat
        lm = (a - rho) @ lhat
        R0sq = t0 * t0 + d * d
        Rp = np.sqrt(lp * lp + R0sq)
        Rm = np.sqrt(lm * lm + R0sq)
        f = _log_ratio(Rp, lp, Rm, lm, R0sq)
        with np.errstate(divide="ignore", invalid="ignore"):
            atp = np.where(R0sq > 0.0, np.arctan2(t0 * lp, R0sq + ad * Rp), 0.0)
            atm = np.where(R0sq > 0.0, np.arctan2(t0 * lm, R0sq + ad * Rm), 0.0)
        omega += atp - atm
        g -= np.outer(f, uhat)
    return g - np.outer(np.sign(d) * omega, n)
