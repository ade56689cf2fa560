"""MFIE Galerkin matrix on RWG functions and the combined-field equation.

Test infrastructure only. The paper solves the sphere (a closed scatterer)
with the combined-field integral equation, linear combination parameter
alpha = 0.6, and defers the operators to its references (Section 2.2). The
reading used here (the usual one): for a closed PEC surface with outward unit
normal n,

    MFIE:  J/2 - n x PV int grad G(r - r') x J(r') dS' = n x H_inc,
    CFIE:  alpha EFIE + (1 - alpha) eta MFIE.

Galerkin testing with f_m gives Z^H_mn = G_mn / 2 - K_mn with the Gram entry
G_mn = int f_m . f_n dS and (since f . (n x X) = (f x n) . X)

    K_mn = int_Tm (f_m x n) . int_Tn grad G(r - r') x f_n(r') dS' dS,

and the tested right-hand side eta <f_m, n x H_inc> = <f_m, n x (k_hat x E_inc)>
for a plane wave (eta H_inc = k_hat x E_inc). The combined system is

    Z^C = alpha Z^E + (1 - alpha) eta Z^H,   V^C = alpha V^E + (1 - alpha) V^H.

Per pair of triangles (T, T') with free vertices v_i, v'_j and RWG factors
c = s l / (2 A): because grad G(r - r') is parallel to r - r', the source
factor (r' - v'_j) may be replaced by (r - v'_j), so the inner integral is one
vector J(r) = int_T' grad_r G(r - r') dS' and

    K_ij = int_T [(r - v_i) x n_T] . [J(r) x (r - v'_j)] dS.

For coplanar T and T' (in particular T = T') every K_ij is zero: J, r - v_i
and r - v'_j then lie in the common plane (the principal value drops the
normal jump of J), so J x (r - v'_j) is normal to it and (r - v_i) x n lies in
it. Such pairs are set to zero exactly. Otherwise both integrals use the
7-point rule, except when T and T' share a vertex: then the first two terms
of grad G's expansion in R,

    grad G = -(r - r')/(4 pi R^3) - k^2 (r - r')/(8 pi R) + S(r - r'),

are integrated in closed form (``potentials.triangle_gradient`` and the
vector potential Iv = int (r' - r)/R), and the remainder
S(d) = (d/R) k^2/(4 pi) phi(kR), phi(x) = (1 - (1 + j x) exp(-j x))/x^2 + 1/2
= j x/3 + x^2/8 - j x^3/30 - x^4/144 + ..., which is smooth (S -> j k^3 d/(12 pi)),
by the 7-point rule (the series below x = 1e-2). The Gram entries use the
7-point rule, exact for the quadratic integrand.
"""

from __future__ import annotations

import math

import numpy as np

from . import quadrature as quad
from .constants import ETA0
from .excitation import unit_vectors
from .mom import dense_z
from .potentials import triangle_gradient, triangle_potentials
from .rwg import RWG

_W = quad.WEIGHTS
_COPLANAR_TOL = 1e-12


def normals(rwg: RWG) -> np.ndarray:
    """Unit normal of each triangle from its vertex order, (v1 - v0) x (v2 - v0)."""
    v = rwg.verts[rwg.tris]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    return n / np.linalg.norm(n, axis=1)[:, None]


def _grad_green(k, d):
    """grad_r G at r - r' = d (..., 3); zero where d = 0."""
    R = np.linalg.norm(d, axis=-1)
    out = np.zeros(d.shape, dtype=np.complex128)
    nz = R > 0
    Rn = R[nz]
    # d/dR exp(-jkR)/(4 pi R) = -(1 + jkR) exp(-jkR) / (4 pi R^2)
    gp = -(1.0 + 1j * k * Rn) * np.exp(-1j * k * Rn) / (4 * math.pi * Rn * Rn)
    out[nz] = (gp / Rn)[:, None] * d[nz]
    return out


def _grad_remainder(k, d):
    """S(d) = grad G + d/(4 pi R^3) + k^2 d/(8 pi R) at d = r - r' (..., 3); zero at d = 0."""
    R = np.linalg.norm(d, axis=-1)
    x = k * R
    phi = np.empty(R.shape, dtype=np.complex128)
    small = x < 1e-2
    xs = x[small]
    phi[small] = 1j * xs / 3 + xs**2 / 8 - 1j * xs**3 / 30 - xs**4 / 144
    xl = x[~small]
    phi[~small] = (1.0 - (1.0 + 1j * xl) * np.exp(-1j * xl)) / (xl * xl) + 0.5
    out = np.zeros(d.shape, dtype=np.complex128)
    nz = R > 0
    out[nz] = (k * k / (4 * math.pi) * phi[nz] / R[nz])[:, None] * d[nz]
    return out


def inner_gradient(k: float, TP: np.ndarray, aTP: float, r: np.ndarray, touching: bool) -> np.ndarray:
    """J(r) = int over TP of grad_r G(r - r') dS' at points r (P, 3)."""
    rq = quad.points(TP)  # (7, 3)
    d = r[:, None, :] - rq[None, :, :]
    if not touching:
        return aTP * np.einsum("q,pqc->pc", _W, _grad_green(k, d))
    _, Iv = triangle_potentials(TP, r)
    return (triangle_gradient(TP, r) / (4 * math.pi) + (k * k / (8 * math.pi)) * Iv
            + aTP * np.einsum("q,pqc->pc", _W, _grad_remainder(k, d)))


def _coplanar(T, TP):
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n = n / np.linalg.norm(n)
    scale = max(np.linalg.norm(T[1] - T[0]), np.linalg.norm(TP[1] - TP[0]))
    return bool(np.all(np.abs((TP - T[0]) @ n) <= _COPLANAR_TOL * scale))


def k_local(rwg: RWG, k: float, t: int, tp: int) -> np.ndarray:
    """K_ij (3, 3) for test triangle t and source triangle tp."""
    V = rwg.verts
    T = V[rwg.tris[t]]
    TP = V[rwg.tris[tp]]
    if t == tp or _coplanar(T, TP):
        return np.zeros((3, 3), dtype=np.complex128)
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n = n / np.linalg.norm(n)
    rp = quad.points(T)
    touching = bool(np.isin(rwg.tris[tp], rwg.tris[t]).any())
    J = inner_gradient(k, TP, rwg.area[tp], rp, touching)  # (7, 3)
    out = np.empty((3, 3), dtype=np.complex128)
    for i in range(3):
        tvec = np.cross(rp - T[i], n)  # (7, 3)
        for j in range(3):
            val = np.einsum("pc,pc->p", tvec, np.cross(J, rp - TP[j]))
            out[i, j] = rwg.area[t] * np.dot(_W, val)
    return out


def k_rows(rwg: RWG, k: float, t: int, tps: np.ndarray) -> np.ndarray:
    """K_ij for test triangle t against source triangles tps, (len(tps), 3, 3):
    the same values as ``k_local``, with the plain 7-point pairs vectorised."""
    tps = np.asarray(tps, dtype=np.int64)
    V = rwg.verts
    T = V[rwg.tris[t]]
    TP = V[rwg.tris[tps]]  # (S, 3, 3)
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n = n / np.linalg.norm(n)
    rp = quad.points(T)  # (7, 3)
    rq = quad.points(TP)  # (S, 7, 3)
    scale = np.linalg.norm(T[1] - T[0])
    coplanar = np.all(np.abs((TP - T[0]) @ n) <= _COPLANAR_TOL * np.maximum(
        scale, np.linalg.norm(TP[:, 1] - TP[:, 0], axis=1))[:, None], axis=1)
    touching = np.isin(rwg.tris[tps], rwg.tris[t]).any(axis=1)
    d = rp[None, :, None, :] - rq[:, None, :, :]  # (S, 7p, 7q, 3)
    J = rwg.area[tps][:, None, None] * np.einsum("q,spqc->spc", _W, _grad_green(k, d))
    for s_ in np.flatnonzero(touching & ~coplanar):
        J[s_] = inner_gradient(k, TP[s_], rwg.area[tps[s_]], rp, True)
    tvec = np.cross(rp[None, :, :] - T[:, None, :], n)  # (i, p, 3)
    src = rp[None, None, :, :] - TP[:, :, None, :]  # (S, j, p, 3)
    cr = np.cross(J[:, None, :, :], src)  # (S, j, p, 3)
    out = rwg.area[t] * np.einsum("p,ipc,sjpc->sij", _W, tvec, cr)
    out[coplanar] = 0.0
    return out


def gram_local(rwg: RWG, t: int) -> np.ndarray:
    """int_T (r - v_i) . (r - v_j) dS, (3, 3)."""
    T = rwg.verts[rwg.tris[t]]
    rp = quad.points(T)
    a = rp[None, :, :] - T[:, None, :]  # (i, p, c)
    return rwg.area[t] * np.einsum("p,ipc,jpc->ij", _W, a, a)


def _tri_coef(rwg: RWG):
    tb = rwg.tri_basis
    tc = np.where(tb >= 0, rwg.tri_sign * rwg.length[np.maximum(tb, 0)] / (2.0 * rwg.area[:, None]), 0.0)
    return tb, tc


def zh_entries(rwg: RWG, k: float, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Z^H_mn = G_mn / 2 - K_mn for individual (m, n) pairs."""
    tb, tc = _tri_coef(rwg)
    out = np.zeros(len(rows), dtype=np.complex128)
    cache = {}
    for idx, (m, n) in enumerate(zip(rows, cols)):
        acc = 0.0 + 0.0j
        for tm in (int(rwg.tplus[m]), int(rwg.tminus[m])):
            im = int(np.flatnonzero(tb[tm] == m)[0])
            for tn in (int(rwg.tplus[n]), int(rwg.tminus[n])):
                jn = int(np.flatnonzero(tb[tn] == n)[0])
                key = (tm, tn)
                if key not in cache:
                    loc = -k_local(rwg, k, tm, tn)
                    if tm == tn:
                        loc = loc + 0.5 * gram_local(rwg, tm)
                    cache[key] = loc
                acc += tc[tm, im] * tc[tn, jn] * cache[key][im, jn]
        out[idx] = acc
    return out


def sparse_zh(rwg: RWG, k: float, indptr: np.ndarray, indices: np.ndarray) -> np.ndarray:
    """Z^H_mn on a CSR pattern (rows m, columns n), values aligned with
    ``indices``; assembled per test triangle over the source triangles its
    rows need."""
    tb, tc = _tri_coef(rwg)
    vals = np.zeros(indices.shape[0], dtype=np.complex128)
    for t in range(rwg.tris.shape[0]):
        rows = tb[t][tb[t] >= 0]
        if rows.size == 0:
            continue
        cols = np.unique(np.concatenate([indices[indptr[m]:indptr[m + 1]] for m in rows]))
        src = np.unique(np.concatenate([rwg.tplus[cols], rwg.tminus[cols]]))
        L = -k_rows(rwg, k, t, src)
        here = np.flatnonzero(src == t)
        if here.size:
            L[here[0]] += 0.5 * gram_local(rwg, t)
        for i in range(3):
            m = tb[t, i]
            if m < 0:
                continue
            lo, hi = indptr[m], indptr[m + 1]
            ncol = indices[lo:hi]
            for side in (rwg.tplus, rwg.tminus):
                tn = side[ncol]
                pos = np.searchsorted(src, tn)
                jn = np.argmax(tb[tn] == ncol[:, None], axis=1)
                vals[lo:hi] += tc[t, i] * tc[tn, jn] * L[pos, i, jn]
    return vals


def dense_zh(rwg: RWG, k: float) -> np.ndarray:
    """Full N x N MFIE matrix Z^H (small closed meshes only), assembled over
    triangle pairs."""
    N = rwg.n
    nt = rwg.tris.shape[0]
    tb, tc = _tri_coef(rwg)
    Z = np.zeros((N, N), dtype=np.complex128)
    all_t = np.arange(nt)
    mask = tb >= 0
    for t in range(nt):
        L = -k_rows(rwg, k, t, all_t)  # (nt, 3, 3)
        L[t] += 0.5 * gram_local(rwg, t)
        for i in range(3):
            if tb[t, i] < 0:
                continue
            vals = tc[t, i] * tc * L[:, i, :]  # (nt, 3)
            np.add.at(Z[tb[t, i]], tb[mask], vals[mask])
    return Z


def dense_zc(rwg: RWG, k: float, alpha: float) -> np.ndarray:
    """Combined-field matrix alpha Z^E + (1 - alpha) eta Z^H."""
    return alpha * dense_z(rwg, k) + (1.0 - alpha) * ETA0 * dense_zh(rwg, k)


def planewave_rhs_h(rwg: RWG, k: float, theta: float, phi: float, pol: int) -> np.ndarray:
    """V^H_m = int f_m . n x (k_hat x E_inc) dS (eta times the tested n x H_inc)."""
    r_hat, th_hat, ph_hat = unit_vectors(theta, phi)
    k_hat = -r_hat
    p_hat = th_hat if pol == 0 else ph_hat
    h_dir = np.cross(k_hat, p_hat)
    nrm = normals(rwg)
    V = np.zeros(rwg.n, dtype=np.complex128)
    for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
        tri = rwg.verts[rwg.tris[side]]
        pts = quad.points(tri)  # (N, 7, 3)
        a = rwg.area[side]
        f = sgn * (rwg.length / (2.0 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
        nxh = np.cross(nrm[side], h_dir)  # (N, 3)
        e = np.exp(-1j * k * (pts @ k_hat))
        V += a * np.einsum("p,np,np->n", quad.WEIGHTS, np.einsum("npc,nc->np", f, nxh), e)
    return V


def planewave_rhs_c(rwg: RWG, k: float, theta: float, phi: float, pol: int, alpha: float) -> np.ndarray:
    from .excitation import planewave_rhs

    return (alpha * planewave_rhs(rwg, k, theta, phi, pol)
            + (1.0 - alpha) * planewave_rhs_h(rwg, k, theta, phi, pol))
