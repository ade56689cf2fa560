"""Adaptive integral method operator: plain FP64 definition.

Test infrastructure only. The paper runs AIM (its refs [2]-[4];
Bleszynski, Bleszynski & Jaroszewicz, Radio Science 1996) with moment
matching on a regular auxiliary grid and a near-zone correction of size set
by gamma = 3 (Section 2.2); each solver iteration applies projection, an FFT
propagation step on the doubled (zero-padded) grid and interpolation, plus the
near-zone correction (Section 4.1 and its footnote on the projection and
interpolation steps). The paper does not write these operators out; this
module states the standard formulation, with the readings taken where the
paper is silent:

Grid. Spacing h; per dimension N_d = max(ceil(extent_d/h - 1e-9) + 1, M + 1)
  nodes centred on the bounding-box centre, x_i = c_d + (i - (N_d - 1)/2) h.
Stencil. Each basis n gets an (M+1)^3 node stencil whose lowest corner
  (the anchor) per dimension is round-half-up((c_n - x_0)/h) - M/2 for even
  M (floor(.) - (M-1)/2 for odd M), clamped into the grid; c_n is the basis
  centre.
Projection Lambda. Tensor-product Lagrange interpolation on the stencil,
  integrated against the basis with the 7-point rule:
      Lambda[n, q, u] = sum_{T in T+-} A_T sum_p w_p F_nq(r_p) l_u(r_p),
  for q = x, y, z (components of f_n) and q = d (div f_n). This matches every
  moment (r - c)^alpha with 0 <= alpha_x, alpha_y, alpha_z <= M exactly (the
  paper matches moments up to third order; the configured order is M = 2).
Grid Green's function. g(u - v) = G(h |u - v|) for u != v and g(0) = 0.
Far operator. Z^grid = j k eta [ sum_{q=x,y,z} Lambda_q^T g Lambda_q
  - k^-2 Lambda_d^T g Lambda_d ].
Near zone. N = {(m, n): |c_m - c_n| <= r_near} (diagonal included) with
  r_near = gamma h; Z^near = Z^MOM - Z^grid on N.
Product. y = Z^near x + j k eta [ sum_q Lambda_q^T (g * Lambda_q x)
  - k^-2 Lambda_d^T (g * Lambda_d x) ], where * is the discrete convolution
  over grid nodes: ``matvec_direct`` sums it directly over occupied nodes,
  ``matvec_fft`` evaluates it by zero-padded FFTs of any size P_d >= 2N_d - 1.
Combined field (closed scatterers, Section 2.2: CFIE with alpha = 0.6; the
  equations are in ``mfie``). The MFIE operator tests the curl of the vector
  potential A_e = g * Lambda_e x (e = x, y, z), which the grid already holds,
  with t_m = f_m x n: its interpolant's curl gives the curl weights
      W[m, e, u] = sum_{T in T+-} A_T sum_p w_p (t_m(r_p) x grad l_u(r_p))_e,
  exact (with the 7-point rule) for fields of tensor degree <= M. Then
      Z^grid = alpha j k eta [ ... as above ... ] - (1 - alpha) eta W^T g Lambda,
  Z^near = alpha Z^E,MOM + (1 - alpha) eta Z^H,MOM - Z^grid, and the product
  interpolates alpha j k eta [ ... ] - (1 - alpha) eta sum_e W_e^T phi_e from
  the same four propagated grids.

FFT thread count follows ``scipy.fft.set_workers`` (default: one worker).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft
import scipy.sparse
from scipy.spatial import cKDTree

from . import quadrature as quad
from .constants import ETA0
from .mfie import normals, sparse_zh
from .mom import sparse_z
from .rwg import RWG


@dataclasses.dataclass
class Grid:
    h: float
    order: int
    n: np.ndarray  # (3,) nodes per dimension
    x0: np.ndarray  # (3,) coordinate of node 0

    @property
    def K(self) -> int:
        return (self.order + 1) ** 3


def grid_plan(verts: np.ndarray, h: float, order: int) -> Grid:
    lo = verts.min(axis=0)
    hi = verts.max(axis=0)
    ext = hi - lo
    n = np.array([max(int(math.ceil(e / h - 1e-9)) + 1, order + 1) for e in ext], dtype=np.int64)
    c = 0.5 * (hi + lo)
    x0 = c - 0.5 * (n - 1) * h
    return Grid(h=h, order=order, n=n, x0=x0)


def anchors(grid: Grid, centres: np.ndarray) -> np.ndarray:
    M = grid.order
    t = (centres - grid.x0) / grid.h
    if M % 2 == 0:
        a = np.floor(t + 0.5).astype(np.int64) - M // 2
    else:
        a = np.floor(t).astype(np.int64) - (M - 1) // 2
    return np.clip(a, 0, grid.n - M - 1)


def lagrange_1d(xi: np.ndarray, M: int) -> np.ndarray:
    """l_s(xi) for nodes 0..M at local coordinate xi: (..., M+1)."""
    out = np.ones(xi.shape + (M + 1,))
    for s in range(M + 1):
        for r in range(M + 1):
            if r != s:
                out[..., s] *= (xi - r) / (s - r)
    return out


def stencil_weights(grid: Grid, anchor: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Tensor Lagrange weights l_u(r) for points pts (..., 3) relative to
    anchors (..., 3): (..., K) with u = (i (M+1) + j)(M+1) + k."""
    M = grid.order
    xi = (pts - grid.x0) / grid.h - anchor
    lx = lagrange_1d(xi[..., 0], M)
    ly = lagrange_1d(xi[..., 1], M)
    lz = lagrange_1d(xi[..., 2], M)
    w = lx[..., :, None, None] * ly[..., None, :, None] * lz[..., None, None, :]
    return w.reshape(w.shape[:-3] + (grid.K,))


def lagrange_1d_deriv(xi: np.ndarray, M: int) -> np.ndarray:
    """d l_s / d xi for nodes 0..M at local coordinate xi: (..., M+1)."""
    out = np.zeros(xi.shape + (M + 1,))
    for s in range(M + 1):
        for j in range(M + 1):  # product rule: drop factor j
            if j == s:
                continue
            term = np.full(xi.shape, 1.0 / (s - j))
            for r in range(M + 1):
                if r != s and r != j:
                    term = term * (xi - r) / (s - r)
            out[..., s] += term
    return out


def stencil_gradients(grid: Grid, anchor: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """grad l_u at points pts (..., 3) for stencils at anchors (..., 3):
    (..., K, 3) with u = (i (M+1) + j)(M+1) + k, in 1/metres."""
    M = grid.order
    xi = (pts - grid.x0) / grid.h - anchor
    L = [lagrange_1d(xi[..., c], M) for c in range(3)]
    D = [lagrange_1d_deriv(xi[..., c], M) / grid.h for c in range(3)]
    gx = D[0][..., :, None, None] * L[1][..., None, :, None] * L[2][..., None, None, :]
    gy = L[0][..., :, None, None] * D[1][..., None, :, None] * L[2][..., None, None, :]
    gz = L[0][..., :, None, None] * L[1][..., None, :, None] * D[2][..., None, None, :]
    g = np.stack([gx, gy, gz], axis=-1)
    return g.reshape(g.shape[:-4] + (grid.K, 3))


def curl_projection(rwg: RWG, grid: Grid, anc: np.ndarray) -> np.ndarray:
    """W[n, e, u] = int over T+- of (t_n x grad l_u)_e dS with t_n = f_n x n_T,
    by the 7-point rule: (N, 3, K) float64."""
    N = rwg.n
    W = np.zeros((N, 3, grid.K))
    nrm = normals(rwg)
    for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
        tri = rwg.verts[rwg.tris[side]]
        pts = quad.points(tri)  # (N, 7, 3)
        a = rwg.area[side]
        F = sgn * (rwg.length / (2.0 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
        t = np.cross(F, nrm[side][:, None, :])  # (N, 7, 3)
        gl = stencil_gradients(grid, anc[:, None, :], pts)  # (N, 7, K, 3)
        c = np.cross(t[:, :, None, :], gl)  # (N, 7, K, 3)
        aw = a[:, None] * quad.WEIGHTS[None, :]
        W += np.einsum("np,npue->neu", aw, c)
    return W


def projection(rwg: RWG, grid: Grid, anc: np.ndarray) -> np.ndarray:
    """Lambda[n, q, u], q in (x, y, z, d): (N, 4, K) float64."""
    N = rwg.n
    lam = np.zeros((N, 4, grid.K))
    for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
        tri = rwg.verts[rwg.tris[side]]
        pts = quad.points(tri)  # (N, 7, 3)
        a = rwg.area[side]
        F = sgn * (rwg.length / (2.0 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
        div = sgn * rwg.length / a  # (N,)
        L = stencil_weights(grid, anc[:, None, :], pts)  # (N, 7, K)
        aw = a[:, None] * quad.WEIGHTS[None, :]  # (N, 7)
        lam[:, 0:3, :] += np.einsum("np,npc,npu->ncu", aw, F, L)
        lam[:, 3, :] += np.einsum("np,n,npu->nu", aw, div, L)
    return lam


def node_offsets(grid: Grid) -> np.ndarray:
    """Integer (i, j, k) offsets of the stencil nodes, in u order: (K, 3)."""
    r = np.arange(grid.order + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)


def grid_green(k: float, h: float, d: np.ndarray) -> np.ndarray:
    """g at integer offsets d (..., 3); g(0) = 0."""
    rho = np.sqrt(np.sum(d.astype(np.float64) ** 2, axis=-1))
    out = np.zeros(rho.shape, dtype=np.complex128)
    nz = rho > 0
    R = h * rho[nz]
    out[nz] = np.exp(-1j * k * R) / (4 * math.pi * R)
    return out


def near_pairs(centres: np.ndarray, r_near: float):
    """CSR (indptr, indices) of {(m, n): |c_m - c_n|^2 <= r_near^2}, columns sorted."""
    N = centres.shape[0]
    tree = cKDTree(centres)
    cand = tree.query_pairs(r_near * (1.0 + 1e-9) + 1e-300, output_type="ndarray")
    m = cand[:, 0]
    n = cand[:, 1]
    d = centres[m] - centres[n]
    keep = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]) <= r_near * r_near
    m = m[keep]
    n = n[keep]
    rows = np.concatenate([m, n, np.arange(N)])
    cols = np.concatenate([n, m, np.arange(N)])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, cols.astype(np.int64)


def zgrid_entries(k: float, grid: Grid, lam: np.ndarray, anc: np.ndarray,
                  rows: np.ndarray, cols: np.ndarray, curl: np.ndarray | None = None,
                  alpha: float = 1.0) -> np.ndarray:
    """Z^grid_mn for pairs (rows[i], cols[i]), grouped by anchor offset; with
    curl weights, the combined-field form."""
    off = node_offsets(grid)
    out = np.zeros(rows.shape[0], dtype=np.complex128)
    delta = anc[rows] - anc[cols]
    key = np.ascontiguousarray(delta).view([("a", np.int64), ("b", np.int64), ("c", np.int64)]).ravel()
    uniq, inv = np.unique(key, return_inverse=True)
    pref = 1j * k * ETA0
    for g_i in range(uniq.shape[0]):
        sel = np.flatnonzero(inv == g_i)
        dlt = delta[sel[0]]
        Gb = grid_green(k, grid.h, dlt[None, None, :] + off[:, None, :] - off[None, :, :])  # (K, K)
        Lm = lam[rows[sel]]  # (P, 4, K)
        Ln = lam[cols[sel]]
        t = np.einsum("uv,pqv->pqu", Gb, Ln)  # (P, 4, K)
        s = np.einsum("pqu,pqu->pq", Lm, t)  # (P, 4)
        out[sel] = pref * (s[:, 0] + s[:, 1] + s[:, 2] - s[:, 3] / k**2)
        if curl is not None:
            kt = np.einsum("peu,peu->p", curl[rows[sel]], t[:, :3, :])
            out[sel] = alpha * out[sel] - (1.0 - alpha) * ETA0 * kt
    return out


@dataclasses.dataclass
class AIMOperator:
    rwg: RWG
    k: float
    grid: Grid
    anc: np.ndarray  # (N, 3)
    lam: np.ndarray  # (N, 4, K)
    near: scipy.sparse.csr_matrix  # Z^near
    zmom_diag: np.ndarray  # diag of Z^MOM (Jacobi preconditioner)
    curl: np.ndarray | None = None  # (N, 3, K) curl weights (combined field only)
    alpha: float = 1.0  # combined-field parameter (1: EFIE)

    @property
    def n(self) -> int:
        return self.rwg.n


def build_operator(rwg: RWG, k: float, h: float, order: int, r_near: float,
                   cfie_alpha: float | None = None) -> AIMOperator:
    """The AIM operator of the EFIE, or with ``cfie_alpha`` of the combined
    field equation alpha EFIE + (1 - alpha) eta MFIE (closed meshes)."""
    grid = grid_plan(rwg.verts, h, order)
    anc = anchors(grid, rwg.centre)
    lam = projection(rwg, grid, anc)
    indptr, indices = near_pairs(rwg.centre, r_near)
    rows = np.repeat(np.arange(rwg.n), np.diff(indptr))
    zmom = sparse_z(rwg, k, indptr, indices)
    curl, alpha = None, 1.0
    if cfie_alpha is not None:
        alpha = float(cfie_alpha)
        curl = curl_projection(rwg, grid, anc)
        zmom = alpha * zmom + (1.0 - alpha) * ETA0 * sparse_zh(rwg, k, indptr, indices)
    zgrid = zgrid_entries(k, grid, lam, anc, rows, indices, curl, alpha)
    near = scipy.sparse.csr_matrix((zmom - zgrid, indices, indptr), shape=(rwg.n, rwg.n))
    diag = zmom[rows == indices]
    return AIMOperator(rwg=rwg, k=k, grid=grid, anc=anc, lam=lam, near=near, zmom_diag=diag,
                       curl=curl, alpha=alpha)


def _node_index(grid: Grid, anc: np.ndarray) -> np.ndarray:
    """Linear grid index (x slowest, z fastest) of each stencil node: (N, K)."""
    nodes = anc[:, None, :] + node_offsets(grid)[None, :, :]
    return (nodes[..., 0] * grid.n[1] + nodes[..., 1]) * grid.n[2] + nodes[..., 2]


def anterpolate(op: AIMOperator, x: np.ndarray) -> np.ndarray:
    """Projection step: source grids s_q = Lambda_q x, dense (R, 4, Nx*Ny*Nz)."""
    x = np.atleast_2d(x)
    V0 = int(np.prod(op.grid.n))
    idx = _node_index(op.grid, op.anc)  # (N, K)
    s = np.zeros((x.shape[0], 4, V0), dtype=np.complex128)
    for r in range(x.shape[0]):
        for q in range(4):
            np.add.at(s[r, q], idx.ravel(), (op.lam[:, q, :] * x[r][:, None]).ravel())
    return s


def interpolate(op: AIMOperator, phi: np.ndarray) -> np.ndarray:
    """Interpolation step: y^far = j k eta [sum_q Lambda_q^T phi_q - k^-2 Lambda_d^T phi_d]
    (combined field: alpha times that, minus (1 - alpha) eta sum_e W_e^T phi_e)."""
    idx = _node_index(op.grid, op.anc)
    k = op.k
    out = np.zeros((phi.shape[0], op.n), dtype=np.complex128)
    for r in range(phi.shape[0]):
        acc = np.zeros(op.n, dtype=np.complex128)
        for q in range(3):
            acc += np.sum(op.lam[:, q, :] * phi[r, q][idx], axis=1)
        acc -= np.sum(op.lam[:, 3, :] * phi[r, 3][idx], axis=1) / k**2
        out[r] = 1j * k * ETA0 * acc
        if op.curl is not None:
            kt = np.zeros(op.n, dtype=np.complex128)
            for e in range(3):
                kt += np.sum(op.curl[:, e, :] * phi[r, e][idx], axis=1)
            out[r] = op.alpha * out[r] - (1.0 - op.alpha) * ETA0 * kt
    return out


def convolve_direct(op: AIMOperator, s: np.ndarray) -> np.ndarray:
    """phi(u) = sum_v g(u - v) s(v), summed directly over occupied nodes."""
    g = op.grid
    occ = np.unique(_node_index(g, op.anc))
    ijk = np.stack(np.unravel_index(occ, tuple(g.n)), axis=1)
    phi = np.zeros_like(s)
    chunk = max(1, 2_000_000 // occ.shape[0])
    for a in range(0, occ.shape[0], chunk):
        G = grid_green(op.k, g.h, ijk[a:a + chunk, None, :] - ijk[None, :, :])  # (c, occ)
        for r in range(s.shape[0]):
            for q in range(4):
                phi[r, q, occ[a:a + chunk]] = G @ s[r, q, occ]
    return phi


def green_spectrum(k: float, grid: Grid, pad) -> np.ndarray:
    """FFT of the circulantly embedded g on a P_x x P_y x P_z grid."""
    P = tuple(int(p) for p in pad)
    idx = []
    for d in range(3):
        i = np.arange(P[d])
        fold = np.minimum(i, P[d] - i)
        valid = fold < grid.n[d]
        idx.append((fold, valid))
    I, J, K = np.meshgrid(idx[0][0], idx[1][0], idx[2][0], indexing="ij")
    V = idx[0][1][:, None, None] & idx[1][1][None, :, None] & idx[2][1][None, None, :]
    gemb = grid_green(k, grid.h, np.stack([I, J, K], axis=-1))
    gemb[~V] = 0.0
    return scipy.fft.fftn(gemb)


def convolve_fft(op: AIMOperator, s: np.ndarray, pad=None, ghat=None) -> np.ndarray:
    g = op.grid
    n = tuple(int(v) for v in g.n)
    if pad is None:
        pad = tuple(2 * v for v in n)
    if ghat is None:
        ghat = green_spectrum(op.k, g, pad)
    phi = np.zeros_like(s)
    for r in range(s.shape[0]):
        for q in range(4):
            S = scipy.fft.fftn(s[r, q].reshape(n), s=pad)
            out = scipy.fft.ifftn(S * ghat)
            phi[r, q] = out[:n[0], :n[1], :n[2]].ravel()
    return phi


def matvec_direct(op: AIMOperator, x: np.ndarray) -> np.ndarray:
    x2 = np.atleast_2d(x)
    y = interpolate(op, convolve_direct(op, anterpolate(op, x2))) + (op.near @ x2.T).T
    return y.reshape(np.shape(x))


def matvec_fft(op: AIMOperator, x: np.ndarray, pad=None, ghat=None) -> np.ndarray:
    x2 = np.atleast_2d(x)
    y = interpolate(op, convolve_fft(op, anterpolate(op, x2), pad, ghat)) + (op.near @ x2.T).T
    return y.reshape(np.shape(x))
