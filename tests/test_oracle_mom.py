"""Pins for the EFIE moment matrix, the excitation and the far field."""

import math

import numpy as np
import pytest

from oracle import excitation, farfield, mie, mom
from oracle import quadrature as quad
from oracle.constants import ETA0, wavelength, wavenumber
from oracle.rwg import build_rwg
from tests.test_oracle_potentials import _u_rule, _v_rule
from workloads import plate_mesh, sphere_mesh

F = 0.3e9
K = wavenumber(F)


def _inner_duffy(TP, r, kern):
    """int_T' kern(R) dS' and int_T' (r' - r) kern(R) dS' by Duffy quadrature."""
    v0, v1, v2 = TP
    n = np.cross(v1 - v0, v2 - v0)
    n /= np.linalg.norm(n)
    d = np.dot(r - v0, n)
    rho = r - d * n
    u, wu = _u_rule()
    v, wv = _v_rule()
    s = 0.0 + 0.0j
    sv = np.zeros(3, dtype=complex)
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        jac = np.dot(np.cross(a - rho, b - rho), n)
        U, Vv = np.meshgrid(u, v, indexing="ij")
        W = np.outer(wu, wv) * U * jac
        pts = rho + U[..., None] * ((a - rho) + Vv[..., None] * (b - a))
        diff = pts - r
        Kv = kern(np.linalg.norm(diff, axis=-1))
        s += np.sum(W * Kv)
        sv += np.einsum("uv,uvc->c", W * Kv, diff)
    return s, sv


def _inner_seven_point(TP, r, kern):
    pts = quad.points(TP)
    area = 0.5 * np.linalg.norm(np.cross(TP[1] - TP[0], TP[2] - TP[0]))
    diff = pts - r
    Kv = kern(np.linalg.norm(diff, axis=1))
    return area * np.sum(quad.WEIGHTS * Kv), area * np.einsum("p,p,pc->c", quad.WEIGHTS, Kv, diff)


def _static(R):
    return 1.0 / (4 * math.pi * R)


def _remainder(R):
    out = np.full(R.shape, -1j * K / (4 * math.pi), dtype=complex)
    nz = R > 0
    out[nz] = (np.exp(-1j * K * R[nz]) - 1.0) / (4 * math.pi * R[nz])
    return out


def _full(R):
    return np.exp(-1j * K * R) / (4 * math.pi * R)


def _local_reference(T, TP, area_t, inner):
    rp = quad.points(T)
    ref = np.zeros((3, 3), dtype=complex)
    for p in range(7):
        s, sv = inner(rp[p])
        for i in range(3):
            for j in range(3):
                val = np.dot(rp[p] - T[i], sv + (rp[p] - TP[j]) * s) - 4.0 / K**2 * s
                ref[i, j] += area_t * quad.WEIGHTS[p] * val
    return ref


def _touching_pair(m, case):
    t = 40
    if case == "self":
        return t, t
    shared = 2 if case == "edge" else 1
    tp = [s for s in range(m.nt) if s != t and len(set(m.tris[s]) & set(m.tris[t])) == shared][0]
    return t, int(tp)


@pytest.mark.parametrize("case", ["self", "edge", "vertex"])
def test_singular_local_matrix_against_duffy(case):
    """Singularity extraction: the closed-form static part equals a Duffy
    integration of 1/(4 pi R); the remainder uses the 7-point rule. The sum
    also stays within the 7-point rule's error of a Duffy integration of the
    full kernel."""
    m = plate_mesh(1.0, F)
    rwg = build_rwg(m.verts, m.tris)
    t, tp = _touching_pair(m, case)
    I = mom.local_matrices(rwg, K, t, np.array([tp]))[0]
    T = m.verts[m.tris[t]]
    TP = m.verts[m.tris[tp]]

    def split(r):
        s1, v1 = _inner_duffy(TP, r, _static)
        s2, v2 = _inner_seven_point(TP, r, _remainder)
        return s1 + s2, v1 + v2

    ref = _local_reference(T, TP, rwg.area[t], split)
    np.testing.assert_allclose(I, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    full = _local_reference(T, TP, rwg.area[t], lambda r: _inner_duffy(TP, r, _full))
    assert np.abs(I - full).max() < 2e-3 * np.abs(full).max()


def test_regular_entries_symmetric():
    """Entries whose four triangle pairs do not touch are exactly symmetric."""
    m = sphere_mesh(0.5, F, nf=3)
    rwg = build_rwg(m.verts, m.tris)
    Z = mom.dense_z(rwg, K)
    tm = np.stack([rwg.tris[rwg.tplus], rwg.tris[rwg.tminus]], axis=1).reshape(rwg.n, 6)
    touch = np.array([[len(set(tm[a]) & set(tm[b])) > 0 for b in range(rwg.n)] for a in range(rwg.n)])
    far = ~touch
    assert far.sum() > 0.5 * rwg.n ** 2
    rel = np.abs(Z - Z.T)[far].max() / np.abs(Z).max()
    assert rel < 1e-13
    # touching entries differ only by the singular-quadrature asymmetry
    assert np.linalg.norm(Z - Z.T) / np.linalg.norm(Z) < 1e-2


def test_normal_incidence_rhs_closed_form():
    """For k_hat = -z on the z=0 plate, E_inc = x_hat is constant and
    V_m = (l/2) [(c+ - p+) + (p- - c-)] . x_hat exactly."""
    m = plate_mesh(1.0, F)
    rwg = build_rwg(m.verts, m.tris)
    V = excitation.planewave_rhs(rwg, K, 0.0, 0.0, 0)
    cp = rwg.centroid[rwg.tplus] - m.verts[rwg.vplus]
    cm = m.verts[rwg.vminus] - rwg.centroid[rwg.tminus]
    ref = 0.5 * rwg.length * (cp + cm)[:, 0]
    np.testing.assert_allclose(V, ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())


def test_grazing_theta_pol_on_plate_is_zero():
    m = plate_mesh(1.0, F)
    rwg = build_rwg(m.verts, m.tris)
    V = excitation.planewave_rhs(rwg, K, math.pi / 2, 0.0, 0)
    assert np.abs(V).max() < 1e-15


def test_far_field_matches_direct_field_at_large_distance():
    """sigma_tt from the radiation vector equals 4 pi r^2 |E_theta|^2 with
    E_theta integrated directly from the vector-potential field at r = 2e4 lambda
    (transverse far-zone part, -j w mu A)."""
    m = plate_mesh(1.0, F)
    rwg = build_rwg(m.verts, m.tris)
    rng = np.random.default_rng(3)
    I = rng.standard_normal(rwg.n) + 1j * rng.standard_normal(rwg.n)
    th, ph = np.array([0.3, 1.1]), np.array([0.2, 2.5])
    sig = farfield.sigma_tt(rwg, K, I, th, ph)
    lam = wavelength(F)
    for a, t_ in enumerate(th):
        for b, p_ in enumerate(ph):
            r_hat, th_hat, _ = excitation.unit_vectors(t_, p_)
            rr = 2e4 * lam
            obs = rr * r_hat
            A = np.zeros(3, dtype=complex)
            for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
                pts = quad.points(m.verts[m.tris[side]])
                ar = rwg.area[side]
                f = sgn * (rwg.length / (2 * ar))[:, None, None] * (pts - m.verts[free][:, None, :])
                R = np.linalg.norm(obs - pts, axis=2)
                G = np.exp(-1j * K * R) / (4 * math.pi * R)
                A += np.einsum("n,np,npc,np->c", I * ar, np.broadcast_to(quad.WEIGHTS, R.shape), f, G)
            Et = -1j * K * ETA0 * np.dot(th_hat, A)
            assert 4 * math.pi * rr**2 * abs(Et) ** 2 == pytest.approx(sig[a, b], rel=1e-4)


@pytest.mark.slow
def test_dense_mom_sphere_against_mie():
    """Dense EFIE MOM on a 0.5-lambda sphere agrees with the Mie series to
    the ~1% level of the paper's sphere references (Table 2)."""
    lam = wavelength(F)
    m = sphere_mesh(0.5, F, nf=5)
    rwg = build_rwg(m.verts, m.tris)
    Z = mom.dense_z(rwg, K)
    V = excitation.planewave_rhs(rwg, K, 0.0, 0.0, 0)
    I = np.linalg.solve(Z, V)
    th, ph = farfield.rcs_grid(3.0)
    s = farfield.sigma_tt(rwg, K, I, th, ph)
    sm = mie.sigma_tt(K, 0.5 * lam, th, ph)
    assert farfield.err_tt(s, sm, th) < 0.04
    # reciprocity: V_a^T I_b = V_b^T I_a for a symmetric Galerkin matrix
    Vb = excitation.planewave_rhs(rwg, K, 1.0, 0.4, 1)
    Ib = np.linalg.solve(Z, Vb)
    delta = np.linalg.norm(Z - Z.T) / np.linalg.norm(Z)
    lhs, rhs = V @ Ib, Vb @ I
    assert abs(lhs - rhs) <= 10 * delta * abs(lhs) + 1e-12


def _pair_classes(rwg):
    """Per basis pair: 2 = identical or sharing a triangle edge (a common
    triangle or a common edge between their triangles), 1 = only a vertex in
    common, 0 = no common vertex."""
    tri_v = [set(rwg.tris[rwg.tplus[n]]) | set(rwg.tris[rwg.tminus[n]]) for n in range(rwg.n)]
    tri_sets = [[set(rwg.tris[rwg.tplus[n]]), set(rwg.tris[rwg.tminus[n]])] for n in range(rwg.n)]
    cls = np.zeros((rwg.n, rwg.n), dtype=np.int8)
    for a in range(rwg.n):
        for b in range(rwg.n):
            if not (tri_v[a] & tri_v[b]):
                continue
            shared = max(len(s & t) for s in tri_sets[a] for t in tri_sets[b])
            cls[a, b] = 2 if shared >= 2 else 1
    return cls


def test_z_entries_equal_dense_matrix():
    """oracle.mom.z_entries (the near-zone reference of the full-size parity
    tests) equals the dense EFIE matrix entry by entry, on self, edge-touching,
    vertex-touching and separated pairs of a 0.4-lambda sphere."""
    m = sphere_mesh(0.4, F, nf=3, jitter_seed=11)
    rwg = build_rwg(m.verts, m.tris)
    Z = mom.dense_z(rwg, K)
    cls = _pair_classes(rwg)
    rng = np.random.default_rng(5)
    rows, cols = [], []
    diag = rng.choice(rwg.n, 30, replace=False)
    rows += list(diag)
    cols += list(diag)
    for c in (2, 1, 0):
        a, b = np.nonzero(cls == c)
        off = a != b
        a, b = a[off], b[off]
        pick = rng.choice(a.size, 70, replace=False)
        rows += list(a[pick])
        cols += list(b[pick])
    rows, cols = np.array(rows), np.array(cols)
    assert rows.size >= 200
    z = mom.z_entries(rwg, K, rows, cols)
    ref = Z[rows, cols]
    np.testing.assert_allclose(z, ref, rtol=1e-14, atol=1e-14 * np.abs(Z).max())


def _rhat(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi),
                     math.cos(theta)])


def _pol_vector(theta, phi, pol):
    """theta_hat = d r_hat / d theta, phi_hat = (d r_hat / d phi) / sin(theta),
    by central differences of r_hat (independent of the excitation code)."""
    e = 1e-6
    if pol == 0:
        v = (_rhat(theta + e, phi) - _rhat(theta - e, phi)) / (2 * e)
    else:
        v = (_rhat(theta, phi + e) - _rhat(theta, phi - e)) / (2 * e * math.sin(theta))
    return v


OBLIQUE_WAVES = [(0.4, 0.3, 0), (0.4, 0.3, 1), (1.1, 2.2, 0), (1.1, 2.2, 1), (2.3, -0.7, 0),
                 (2.3, -0.7, 1), (2.9, 4.0, 0), (2.9, 4.0, 1)]


def _rhs_reciprocity_errors(rwg):
    """max over waves of max_m |V_m - p_hat . N_m(r_hat)| / max |V|, with N_m
    the radiation vector of the unit current on basis m: a plane wave arriving
    from r_hat has phase exp(-j k k_hat . r) = exp(+j k r_hat . r), the
    radiation vector's kernel, so V_m = p_hat . N_m(r_hat)."""
    errs = []
    for th, ph, pol in OBLIQUE_WAVES:
        V = excitation.planewave_rhs(rwg, K, th, ph, pol)
        p = _pol_vector(th, ph, pol)
        ref = np.empty(rwg.n, dtype=np.complex128)
        for n in range(rwg.n):
            e = np.zeros(rwg.n, dtype=np.complex128)
            e[n] = 1.0
            Nv = farfield.radiation_vector(rwg, K, e, np.array([th]), np.array([ph]))[0, 0]
            ref[n] = p @ Nv
        errs.append(np.abs(V - ref).max() / np.abs(ref).max())
    return max(errs)


@pytest.mark.parametrize("kind", ["sphere", "plate"])
def test_oblique_incidence_rhs_is_radiation_vector(kind):
    """Oblique plane-wave right-hand sides, both polarisations, every basis:
    V_m = p_hat(theta_i, phi_i) . N_m(r_hat(theta_i, phi_i)) (the radiation
    vector is pinned against the direct field above)."""
    m = (sphere_mesh(0.4, F, nf=3, jitter_seed=12) if kind == "sphere"
         else plate_mesh(1.0, F, squares_per_lambda=5, jitter_seed=13))
    rwg = build_rwg(m.verts, m.tris)
    assert _rhs_reciprocity_errors(rwg) < 1e-9


@pytest.mark.parametrize("plant", ["theta_hat", "k_hat"])
def test_oblique_rhs_check_catches_planted_errors(monkeypatch, plant):
    """A sign flip planted in the oracle's unit vectors (theta_hat, or the
    propagation direction k_hat = -r_hat) makes the identity above fail."""
    m = sphere_mesh(0.4, F, nf=2, jitter_seed=12)
    rwg = build_rwg(m.verts, m.tris)
    orig = excitation.unit_vectors

    def planted(theta, phi):
        r, t, p = orig(theta, phi)
        return (r, -t, p) if plant == "theta_hat" else (-r, t, p)

    monkeypatch.setattr(excitation, "unit_vectors", planted)
    assert _rhs_reciprocity_errors(rwg) > 0.1
