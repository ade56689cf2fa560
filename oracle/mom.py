"""EFIE Galerkin moment matrix on RWG functions, with singularity extraction.

Test infrastructure only. The paper solves the electric-field integral
equation for the open plate (Section 2.2) with the method of moments; AIM
accelerates the product with this same matrix (Section 1, refs [1]-[4]). For
RWG testing and basis functions f_m, f_n (Rao-Wilton-Glisson 1982):

    Z_mn = j k eta  int_Tm int_Tn [ f_m . f_n - k^-2 (div f_m)(div' f_n) ] G(|r - r'|) dS' dS

with G(R) = exp(-j k R)/(4 pi R). Per pair of triangles (T, T') with free
vertices v_i of T and v'_j of T', the RWG factors give

    Z_mn += j k eta s_m s_n l_m l_n / (4 A A') * I_ij,
    I_ij = int_T int_T' [ (r - v_i).(r' - v'_j) - 4/k^2 ] G dS' dS.

Both integrals use the 7-point rule, except when T and T' are the same
triangle or share a vertex or an edge. Then the inner integral is split as
G = 1/(4 pi R) + (exp(-j k R) - 1)/(4 pi R): the static part in closed form
(``potentials``), the smooth remainder by the 7-point rule, with its R -> 0
limit -j k / (4 pi) for the scalar kernel and 0 for the (r' - r) kernel.
"""

from __future__ import annotations

import math

import numpy as np

from . import quadrature as quad
from .constants import ETA0
from .potentials import triangle_potentials
from .rwg import RWG

_W = quad.WEIGHTS
_W2 = np.outer(_W, _W)


def _singular_local(k, T, aT, TP, aTP):
    """3x3 local matrix for a touching pair (closed-form static part)."""
    rp = quad.points(T)  # (7,3)
    rq = quad.points(TP)  # (7,3)
    I1, Iv = triangle_potentials(TP, rp)
    d = rq[None, :, :] - rp[:, None, :]  # r' - r, (p, q, 3)
    R = np.linalg.norm(d, axis=2)
    E = np.empty(R.shape, dtype=np.complex128)
    zero = R == 0.0
    E[~zero] = (np.exp(-1j * k * R[~zero]) - 1.0) / R[~zero]
    E[zero] = -1j * k
    J1 = I1 / (4 * math.pi) + aTP * (E @ _W) / (4 * math.pi)  # (p,)
    Jr = Iv / (4 * math.pi) + aTP * np.einsum("q,pq,pqc->pc", _W, E, d) / (4 * math.pi)
    out = np.empty((3, 3), dtype=np.complex128)
    for i in range(3):
        a = rp - T[i]
        for j in range(3):
            inner = Jr + (rp - TP[j]) * J1[:, None]
            val = np.einsum("pc,pc->p", a, inner) - (4.0 / k**2) * J1
            out[i, j] = aT * np.dot(_W, val)
    return out


def local_matrices(rwg: RWG, k: float, t: int, tps: np.ndarray) -> np.ndarray:
    """I_ij for test triangle t against source triangles tps: (len(tps), 3, 3)."""
    tps = np.asarray(tps, dtype=np.int64)
    V = rwg.verts
    T = V[rwg.tris[t]]
    TP = V[rwg.tris[tps]]
    aT = rwg.area[t]
    aTP = rwg.area[tps]
    rp = quad.points(T)
    rq = quad.points(TP)
    A = rp[None, :, :] - T[:, None, :]  # (i, p, c)
    B = rq[:, None, :, :] - TP[:, :, None, :]  # (m, j, q, c)
    R = np.linalg.norm(rp[None, :, None, :] - rq[:, None, :, :], axis=3)  # (m, p, q)
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.exp(-1j * k * R) / (4 * math.pi * R)
    Gw = G * _W2[None]
    I = np.einsum("mpq,ipc,mjqc->mij", Gw, A, B)
    I -= (4.0 / k**2) * Gw.sum(axis=(1, 2))[:, None, None]
    I *= (aT * aTP)[:, None, None]
    shares = (rwg.tris[tps][:, :, None] == rwg.tris[t][None, None, :]).any(axis=(1, 2))
    for s in np.flatnonzero(shares):
        I[s] = _singular_local(k, T, aT, TP[s], aTP[s])
    return I


def _coef(rwg: RWG, k: float, t: int):
    """Per local vertex of t: (basis id, s * l / (2 A)) with -1 where no basis."""
    b = rwg.tri_basis[t]
    c = np.where(b >= 0, rwg.tri_sign[t] * rwg.length[np.maximum(b, 0)] / (2.0 * rwg.area[t]), 0.0)
    return b, c


def dense_z(rwg: RWG, k: float) -> np.ndarray:
    """Full N x N EFIE matrix (small meshes only)."""
    N = rwg.n
    nt = rwg.tris.shape[0]
    Z = np.zeros((N, N), dtype=np.complex128)
    all_t = np.arange(nt)
    tb = rwg.tri_basis
    tc = np.where(tb >= 0, rwg.tri_sign * rwg.length[np.maximum(tb, 0)] / (2.0 * rwg.area[:, None]), 0.0)
    pref = 1j * k * ETA0
    for t in range(nt):
        I = local_matrices(rwg, k, t, all_t)  # (nt, 3, 3)
        bm, cm = _coef(rwg, k, t)
        for i in range(3):
            if bm[i] < 0:
                continue
            vals = pref * cm[i] * tc * I[:, i, :]  # (nt, 3)
            mask = tb >= 0
            np.add.at(Z[bm[i]], tb[mask], vals[mask])
    return Z


def z_entries(rwg: RWG, k: float, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Z_mn for individual (m, n) pairs by summing their four triangle pairs."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.zeros(rows.shape[0], dtype=np.complex128)
    pref = 1j * k * ETA0
    for idx, (m, n) in enumerate(zip(rows, cols)):
        acc = 0.0 + 0.0j
        for tm in (rwg.tplus[m], rwg.tminus[m]):
            im = int(np.flatnonzero(rwg.tri_basis[tm] == m)[0])
            cm = rwg.tri_sign[tm, im] * rwg.length[m] / (2.0 * rwg.area[tm])
            tns = np.array([rwg.tplus[n], rwg.tminus[n]])
            I = local_matrices(rwg, k, int(tm), tns)
            for s, tn in enumerate(tns):
                jn = int(np.flatnonzero(rwg.tri_basis[tn] == n)[0])
                cn = rwg.tri_sign[tn, jn] * rwg.length[n] / (2.0 * rwg.area[tn])
                acc += cm * cn * I[s, im, jn]
        out[idx] = pref * acc
    return out


def sparse_z(rwg: RWG, k: float, indptr: np.ndarray, indices: np.ndarray) -> np.ndarray:
    """Z_mn on a CSR pattern (rows m, columns n), grouped by triangle pairs.

    Returns the values array aligned with ``indices``."""
    vals = np.zeros(indices.shape[0], dtype=np.complex128)
    pref = 1j * k * ETA0
    nt = rwg.tris.shape[0]
    tb = rwg.tri_basis
    tc = np.where(tb >= 0, rwg.tri_sign * rwg.length[np.maximum(tb, 0)] / (2.0 * rwg.area[:, None]), 0.0)
    for t in range(nt):
        bm = tb[t]
        rows = bm[bm >= 0]
        if rows.size == 0:
            continue
        cols = np.unique(np.concatenate([indices[indptr[m]:indptr[m + 1]] for m in rows]))
        src_t = np.unique(np.concatenate([rwg.tplus[cols], rwg.tminus[cols]]))
        I = local_matrices(rwg, k, t, src_t)  # (S, 3, 3)
        cm = tc[t]
        for i in range(3):
            m = bm[i]
            if m < 0:
                continue
            lo, hi = indptr[m], indptr[m + 1]
            ncols = indices[lo:hi]
            acc = np.zeros(hi - lo, dtype=np.complex128)
            for side in (rwg.tplus, rwg.tminus):
                tn = side[ncols]
                pos = np.searchsorted(src_t, tn)
                jn = np.argmax(tb[tn] == ncols[:, None], axis=1)
                acc += tc[tn, jn] * I[pos, i, jn]
            vals[lo:hi] += pref * cm[i] * acc
    return vals
