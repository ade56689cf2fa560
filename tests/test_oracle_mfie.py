"""Pins for the MFIE / combined-field oracle (closed scatterers).

The gradient closed form is checked against central differences of the
(separately pinned) potential I1 and against Duffy quadrature; the touching
pair extraction against subdivided quadrature; the assembled operators
against the Mie series, against special cases with exact answers (coplanar
pairs, the flat plate's right-hand side) and, with the sign of the K term
flipped in the oracle itself, for sensitivity of the Mie pin.
"""

import math

import numpy as np
import pytest

from oracle import excitation, farfield, mfie, mie, mom
from oracle import quadrature as quad
from oracle.constants import ETA0, wavelength, wavenumber
from oracle.potentials import triangle_gradient, triangle_potentials
from oracle.rwg import build_rwg
from tests.test_oracle_potentials import _u_rule, _v_rule
from workloads import plate_mesh, sphere_mesh

F = 0.3e9
K = wavenumber(F)
TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.05]])


def _duffy_gradient(tri, r):
    """int_T grad_r 1/R dS' = -int (r - r')/R^3 dS' by the Duffy map about the
    projection of r (graded Gauss-Legendre rules)."""
    v0, v1, v2 = tri
    n = np.cross(v1 - v0, v2 - v0)
    n /= np.linalg.norm(n)
    d = np.dot(r - v0, n)
    rho = r - d * n
    u, wu = _u_rule()
    v, wv = _v_rule()
    out = np.zeros(3)
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        jac = np.dot(np.cross(a - rho, b - rho), n)
        U, Vv = np.meshgrid(u, v, indexing="ij")
        W = np.outer(wu, wv)
        pts = rho + U[..., None] * ((a - rho) + Vv[..., None] * (b - a))
        diff = r - pts
        R = np.linalg.norm(diff, axis=-1)
        out -= np.einsum("uv,uvc->c", W * U * jac / R**3, diff)
    return out


def _subdivided_points(tri, levels):
    """7-point rule on a 4^levels uniform subdivision: points (P, 3), weights
    (P,) summing to the area."""
    tris = [np.asarray(tri, float)]
    for _ in range(levels):
        nxt = []
        for t in tris:
            a, b, c = t
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array(x) for x in ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca))]
        tris = nxt
    T = np.stack(tris)
    pts = quad.points(T).reshape(-1, 3)
    area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    w = (area[:, None] * quad.WEIGHTS[None, :]).ravel()
    return pts, w


def test_gradient_matches_differences_of_the_potential():
    rng = np.random.default_rng(1)
    r = rng.normal(size=(12, 3)) * 0.6 + np.array([0.4, 0.3, 0.1])
    g = triangle_gradient(TRI, r)
    eps = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = eps
        fd = (triangle_potentials(TRI, r + e)[0] - triangle_potentials(TRI, r - e)[0]) / (2 * eps)
        np.testing.assert_allclose(g[:, c], fd, rtol=0, atol=1e-8 * np.abs(g).max())


@pytest.mark.parametrize("r", [[0.3, 0.3, 0.2], [0.35, 0.3, 0.026], [1.4, 0.2, 0.3], [0.5, -0.2, 0.01]])
def test_gradient_matches_duffy(r):
    r = np.asarray(r)
    np.testing.assert_allclose(triangle_gradient(TRI, r[None])[0], _duffy_gradient(TRI, r),
                               rtol=1e-9, atol=1e-9)


def test_gradient_normal_jump_is_the_solid_angle():
    """Just above and below an interior point the normal component tends to
    -/+ 2 pi (the half-space solid angle) and is zero in the plane."""
    tri = TRI * np.array([1.0, 1.0, 0.0])  # in z = 0, so d = 0 exactly in the plane
    n = np.array([0.0, 0.0, 1.0])
    c = np.array([0.4, 0.3, 0.0])
    up = triangle_gradient(tri, (c + 1e-9 * n)[None])[0] @ n
    dn = triangle_gradient(tri, (c - 1e-9 * n)[None])[0] @ n
    on = triangle_gradient(tri, c[None])[0] @ n
    assert abs(up + 2 * math.pi) < 1e-6 and abs(dn - 2 * math.pi) < 1e-6 and abs(on) < 1e-12


def test_touching_inner_gradient_matches_subdivided_quadrature():
    """The extracted inner integral at points near a triangle (as the outer
    7-point points of an adjacent triangle are) against a 4^7-fold subdivided
    7-point rule of grad G (one extracted term only leaves 1.5e-3)."""
    m = sphere_mesh(0.25, F, nf=2)
    rwg = build_rwg(m.verts, m.tris)
    t = 0
    nb = [s for s in range(rwg.tris.shape[0]) if s != t and np.isin(rwg.tris[s], rwg.tris[t]).any()][0]
    TP = rwg.verts[rwg.tris[t]]
    r = quad.points(rwg.verts[rwg.tris[nb]])
    J = mfie.inner_gradient(K, TP, rwg.area[t], r, True)
    pts, w = _subdivided_points(TP, 7)
    ref = np.einsum("q,pqc->pc", w, mfie._grad_green(K, r[:, None, :] - pts[None, :, :]))
    assert np.abs(J - ref).max() <= 2e-5 * np.abs(ref).max()


def test_remainder_series_meets_the_closed_form():
    """The small-argument series of the remainder and its direct formula agree
    where they switch (kR = 1e-2), and the remainder vanishes like k^3 R."""
    for x in (1e-2 * (1 - 1e-12), 1e-2 * (1 + 1e-12)):
        d = np.array([[x / K, 0.0, 0.0]])
        v = mfie._grad_remainder(K, d)[0, 0]
        ref = 1j * K**3 * d[0, 0] / (12 * math.pi)
        assert abs(v - ref) <= 0.02 * abs(ref)
    a = mfie._grad_remainder(K, np.array([[1e-2 / K * (1 - 1e-12), 0, 0]]))[0, 0]
    b = mfie._grad_remainder(K, np.array([[1e-2 / K * (1 + 1e-12), 0, 0]]))[0, 0]
    assert abs(a - b) <= 1e-9 * abs(a)


def test_gram_is_exact():
    """int_T (r - v_i).(r - v_j) dS against a finely subdivided rule."""
    m = sphere_mesh(0.25, F, nf=2)
    rwg = build_rwg(m.verts, m.tris)
    for t in (0, 7):
        T = rwg.verts[rwg.tris[t]]
        pts, w = _subdivided_points(T, 3)
        a = pts[None, :, :] - T[:, None, :]
        ref = np.einsum("p,ipc,jpc->ij", w, a, a)
        np.testing.assert_allclose(mfie.gram_local(rwg, t), ref, rtol=1e-12, atol=0)


def test_vectorised_rows_equal_the_plain_pair_form():
    m = sphere_mesh(0.25, F, nf=3)
    rwg = build_rwg(m.verts, m.tris)
    nt = rwg.tris.shape[0]
    for t in (0, 11, 40):
        a = mfie.k_rows(rwg, K, t, np.arange(nt))
        b = np.stack([mfie.k_local(rwg, K, t, s) for s in range(nt)])
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_flat_plate_special_cases():
    """Every pair of a flat plate is coplanar, so Z^H is half the Gram matrix
    exactly; with the +z normal and a wave toward -z, n x (k x E) = E, so the
    MFIE right-hand side equals the EFIE one."""
    m = plate_mesh(1.0, F)
    rwg = build_rwg(m.verts, m.tris)
    assert np.allclose(mfie.normals(rwg), [0, 0, 1])
    ZH = mfie.dense_zh(rwg, K)
    G = np.zeros((rwg.n, rwg.n))
    tb, tc = mfie._tri_coef(rwg)
    for t in range(rwg.tris.shape[0]):
        g = mfie.gram_local(rwg, t)
        for i in range(3):
            for j in range(3):
                if tb[t, i] >= 0 and tb[t, j] >= 0:
                    G[tb[t, i], tb[t, j]] += tc[t, i] * tc[t, j] * g[i, j]
    assert np.abs(ZH - 0.5 * G).max() == 0.0
    VE = excitation.planewave_rhs(rwg, K, 0.0, 0.0, 0)
    VH = mfie.planewave_rhs_h(rwg, K, 0.0, 0.0, 0)
    np.testing.assert_allclose(VH, VE, rtol=0, atol=1e-15 * np.abs(VE).max())


@pytest.fixture(scope="module")
def sphere05():
    m = sphere_mesh(0.5, F, nf=4)
    rwg = build_rwg(m.verts, m.tris)
    return m, rwg, mom.dense_z(rwg, K), mfie.dense_zh(rwg, K)


def test_sparse_matches_dense(sphere05):
    from oracle import aim as oaim

    m, rwg, _, ZH = sphere05
    ip, ind = oaim.near_pairs(rwg.centre, 0.3 * m.lam)
    rows = np.repeat(np.arange(rwg.n), np.diff(ip))
    v = mfie.sparse_zh(rwg, K, ip, ind)
    assert np.abs(v - ZH[rows, ind]).max() <= 1e-14 * np.abs(ZH).max()
    e = mfie.zh_entries(rwg, K, rows[:300], ind[:300])
    assert np.abs(e - ZH[rows[:300], ind[:300]]).max() <= 1e-14 * np.abs(ZH).max()


def test_mfie_and_cfie_against_mie(sphere05):
    """EFIE, CFIE (alpha = 0.6, the paper's) and MFIE solutions of a
    0.5-lambda sphere against the Mie series; the MFIE with the sign of its K
    term flipped (a planted oracle mistake) misses by far more."""
    m, rwg, ZE, ZH = sphere05
    th, ph = farfield.rcs_grid(3.0)
    sm = mie.sigma_tt(K, 0.5 * wavelength(F), th, ph)
    VE = excitation.planewave_rhs(rwg, K, 0.0, 0.0, 0)
    VH = mfie.planewave_rhs_h(rwg, K, 0.0, 0.0, 0)
    errs = {}
    for alpha in (1.0, 0.6, 0.0):
        Z = alpha * ZE + (1 - alpha) * ETA0 * ZH
        I = np.linalg.solve(Z, alpha * VE + (1 - alpha) * VH)
        errs[alpha] = farfield.err_tt(farfield.sigma_tt(rwg, K, I, th, ph), sm, th)
    assert errs[1.0] < 0.05 and errs[0.6] < 0.06 and errs[0.0] < 0.12
    Kterm = 0.5 * _gram(rwg) - ZH  # Z^H = G/2 - K
    I = np.linalg.solve(ETA0 * (0.5 * _gram(rwg) + Kterm), VH)  # sign of K flipped
    wrong = farfield.err_tt(farfield.sigma_tt(rwg, K, I, th, ph), sm, th)
    assert wrong > 2 * errs[0.0] and wrong > 0.2


def _gram(rwg):
    G = np.zeros((rwg.n, rwg.n))
    tb, tc = mfie._tri_coef(rwg)
    for t in range(rwg.tris.shape[0]):
        g = mfie.gram_local(rwg, t)
        for i in range(3):
            for j in range(3):
                if tb[t, i] >= 0 and tb[t, j] >= 0:
                    G[tb[t, i], tb[t, j]] += tc[t, i] * tc[t, j] * g[i, j]
    return G
