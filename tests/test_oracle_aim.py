"""Pins for the AIM oracle: projection, grid Green's function, near zone and
the two forms of the product."""

import itertools

import numpy as np
import pytest

from oracle import aim, mom
from oracle import quadrature as quad
from oracle.constants import ETA0, wavelength, wavenumber
from oracle.rwg import build_rwg
from workloads import plate_mesh, random_current, sphere_mesh

F = 0.3e9
K = wavenumber(F)
LAM = wavelength(F)


def _setup(mesh, h=0.1, M=2, rn=0.3):
    rwg = build_rwg(mesh.verts, mesh.tris)
    op = aim.build_operator(rwg, K, h * LAM, M, rn * LAM)
    return rwg, op


@pytest.fixture(scope="module")
def plate():
    return _setup(plate_mesh(1.0, F))


@pytest.fixture(scope="module")
def sphere():
    return _setup(sphere_mesh(0.4, F, nf=3))


def _node_coords(grid, anc):
    off = aim.node_offsets(grid)
    return grid.x0 + grid.h * (anc[:, None, :] + off[None, :, :])  # (N, K, 3)


def _quad_moments(rwg, centre, alpha):
    """sum over T+- of A w F_q (r - c)^alpha, straight from the basis."""
    out = np.zeros((rwg.n, 4))
    for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
        pts = quad.points(rwg.verts[rwg.tris[side]])
        a = rwg.area[side]
        F_ = sgn * (rwg.length / (2 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
        div = sgn * rwg.length / a
        mono = np.prod((pts - centre[:, None, :]) ** np.asarray(alpha), axis=2)
        aw = a[:, None] * quad.WEIGHTS
        out[:, :3] += np.einsum("np,npc,np->nc", aw, F_, mono)
        out[:, 3] += np.einsum("np,n,np->n", aw, div, mono)
    return out


@pytest.mark.parametrize("which", ["plate", "sphere"])
def test_moment_identity(which, plate, sphere):
    """sum_u Lambda_u (r_u - c)^alpha equals the quadrature moment of the
    basis for every tensor index alpha <= M."""
    rwg, op = plate if which == "plate" else sphere
    nodes = _node_coords(op.grid, op.anc)
    c = rwg.centre
    scale = np.abs(op.lam).max()
    for alpha in itertools.product(range(3), repeat=3):
        mono = np.prod((nodes - c[:, None, :]) ** np.asarray(alpha), axis=2)  # (N, K)
        lhs = np.einsum("nqu,nu->nq", op.lam, mono)
        rhs = _quad_moments(rwg, c, alpha)
        h_pow = op.grid.h ** sum(alpha)
        assert np.abs(lhs - rhs).max() <= 1e-12 * scale * h_pow


@pytest.mark.parametrize("M", [1, 3, 4, 5])
def test_moment_identity_other_orders(M):
    """The same identity at every supported stencil order, on a sphere and
    on a jittered plate (up to fifth order: the paper's reference setting)."""
    for mesh in (sphere_mesh(0.4, F, nf=2), plate_mesh(1.0, F, jitter_seed=7)):
        rwg = build_rwg(mesh.verts, mesh.tris)
        grid = aim.grid_plan(rwg.verts, 0.1 * LAM, M)
        anc = aim.anchors(grid, rwg.centre)
        lam = aim.projection(rwg, grid, anc)
        assert lam.shape == (rwg.n, 4, (M + 1) ** 3)
        assert np.all(anc >= 0) and np.all(anc + M < np.asarray(grid.n))
        nodes = _node_coords(grid, anc)
        c = rwg.centre
        scale = np.abs(lam).max()
        for alpha in itertools.product(range(M + 1), repeat=3):
            mono = np.prod((nodes - c[:, None, :]) ** np.asarray(alpha), axis=2)
            lhs = np.einsum("nqu,nu->nq", lam, mono)
            rhs = _quad_moments(rwg, c, alpha)
            assert np.abs(lhs - rhs).max() <= 1e-11 * scale * grid.h ** sum(alpha)
        # one order more is not matched in general (the identity is tight)
        alpha = (M + 1, 0, 0)
        mono = np.prod((nodes - c[:, None, :]) ** np.asarray(alpha), axis=2)
        lhs = np.einsum("nqu,nu->nq", lam, mono)
        rhs = _quad_moments(rwg, c, alpha)
        assert np.abs(lhs - rhs).max() > 1e-6 * scale * grid.h ** (M + 1)


def test_lagrange_equals_vandermonde_solve(sphere):
    """Lambda from Lagrange weights equals the solution of the (M+1)^3
    moment-matching system V^T Lambda = moments."""
    rwg, op = sphere
    nodes = _node_coords(op.grid, op.anc)
    alphas = list(itertools.product(range(3), repeat=3))
    c = rwg.centre
    moments = np.stack([_quad_moments(rwg, c, a) for a in alphas], axis=1)  # (N, 27, 4)
    for n in range(0, rwg.n, 7):
        Vm = np.stack([np.prod(((nodes[n] - c[n]) / op.grid.h) ** np.asarray(a), axis=1) for a in alphas])
        scale = np.array([op.grid.h ** sum(a) for a in alphas])
        sol = np.linalg.solve(Vm, moments[n] / scale[:, None])  # (27, 4)
        np.testing.assert_allclose(sol.T, op.lam[n], rtol=0, atol=1e-11 * np.abs(op.lam[n]).max())


def test_charge_neutral_projection(plate, sphere):
    for rwg, op in (plate, sphere):
        s = op.lam[:, 3, :].sum(axis=1)
        assert np.abs(s).max() < 1e-12 * np.abs(op.lam[:, 3, :]).max()


def test_plate_planar_degeneracy(plate):
    """On the z=0 plate Lambda_z = 0 and the z = +-h stencil planes carry
    exactly zero weight."""
    rwg, op = plate
    assert tuple(op.grid.n) == (11, 11, 3)
    assert np.all(op.anc[:, 2] == 0)
    assert np.all(op.lam[:, 2, :] == 0.0)
    off = aim.node_offsets(op.grid)
    assert np.all(op.lam[:, :, off[:, 2] != 1] == 0.0)


def test_near_zone_brute_force(plate, sphere):
    for rwg, op in (plate, sphere):
        c = rwg.centre
        d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(axis=2)
        ref = d2 <= (0.3 * LAM) ** 2
        got = np.zeros_like(ref)
        rows = np.repeat(np.arange(rwg.n), np.diff(op.near.indptr))
        got[rows, op.near.indices] = True
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("which", ["plate", "sphere"])
def test_fft_equals_direct_sum(which, plate, sphere):
    rwg, op = plate if which == "plate" else sphere
    x = random_current(rwg.n, nrhs=2)
    yd = aim.matvec_direct(op, x)
    yf = aim.matvec_fft(op, x)
    assert np.linalg.norm(yd - yf) <= 1e-12 * np.linalg.norm(yd)
    # any padding P_d >= 2 N_d - 1 gives the same linear convolution
    pad = tuple(int(2 * n - 1 + e) for n, e in zip(op.grid.n, (0, 3, 1)))
    yp = aim.matvec_fft(op, x, pad=pad)
    assert np.linalg.norm(yp - yf) <= 1e-12 * np.linalg.norm(yf)


def test_linear_and_far_part_symmetric(sphere):
    rwg, op = sphere
    x = random_current(rwg.n, nrhs=2, seed=11)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    y = aim.matvec_direct(op, a * x[0] + b * x[1])
    assert np.linalg.norm(y - a * aim.matvec_direct(op, x[0]) - b * aim.matvec_direct(op, x[1])) < 1e-12 * np.linalg.norm(y)
    phi = aim.convolve_direct(op, aim.anterpolate(op, x[:1]))
    yf0 = aim.interpolate(op, phi)[0]
    phi1 = aim.convolve_direct(op, aim.anterpolate(op, x[1:]))
    yf1 = aim.interpolate(op, phi1)[0]
    assert abs(x[1] @ yf0 - x[0] @ yf1) < 1e-12 * abs(x[1] @ yf0)


@pytest.mark.parametrize("mesh", [plate_mesh(2 / 9, F), sphere_mesh(0.15, F, nf=1), sphere_mesh(0.25, F, nf=2)],
                         ids=["plate2x2", "icosahedron", "sphere_nf2"])
def test_aim_equals_mom_when_everything_is_near(mesh):
    """With r_near beyond the scatterer's diameter every pair is near and
    Z^near + Z^grid reproduces Z^MOM to rounding."""
    rwg, op = _setup(mesh, rn=10.0)
    Z = mom.dense_z(rwg, K)
    x = random_current(rwg.n)[0]
    y = aim.matvec_direct(op, x)
    assert np.linalg.norm(y - Z @ x) <= 1e-12 * np.linalg.norm(Z @ x)
    assert op.near.nnz == rwg.n ** 2


def test_grid_green_convention():
    g = aim.grid_green(K, 0.1 * LAM, np.array([[0, 0, 0], [1, 0, 0], [0, 3, 4]]))
    h = 0.1 * LAM
    assert g[0] == 0
    assert g[1] == pytest.approx(np.exp(-1j * K * h) / (4 * np.pi * h), rel=1e-15)
    assert g[2] == pytest.approx(np.exp(-1j * K * 5 * h) / (4 * np.pi * 5 * h), rel=1e-15)


def test_grid_plan_sizes():
    for L, n in ((1.0, 11), (2.0, 21), (16.0, 161)):
        m = plate_mesh(L, 4.8e9)
        g = aim.grid_plan(m.verts, 0.1 * m.lam, 2)
        assert tuple(g.n) == (n, n, 3)


# ---- combined field (closed scatterers) -------------------------------------

@pytest.fixture(scope="module")
def sphere_cfie():
    from oracle import mfie

    mesh = sphere_mesh(0.4, F, nf=3)
    rwg = build_rwg(mesh.verts, mesh.tris)
    ZC = 0.6 * mom.dense_z(rwg, K) + 0.4 * ETA0 * mfie.dense_zh(rwg, K)
    return rwg, ZC


@pytest.mark.parametrize("M", [2, 3])
def test_curl_moment_identity(M):
    """sum_u W_e[u] p(r_u) = int (t x grad p)_e dS, t = f x n, for every
    monomial p = (r - c)^alpha with alpha <= M (gradient taken analytically)."""
    from oracle import mfie

    mesh = sphere_mesh(0.4, F, nf=2)
    rwg = build_rwg(mesh.verts, mesh.tris)
    grid = aim.grid_plan(rwg.verts, 0.1 * LAM, M)
    anc = aim.anchors(grid, rwg.centre)
    W = aim.curl_projection(rwg, grid, anc)
    nodes = _node_coords(grid, anc)
    c = rwg.centre
    nrm = mfie.normals(rwg)
    for alpha in itertools.product(range(M + 1), repeat=3):
        al = np.asarray(alpha)
        lhs = np.einsum("neu,nu->ne", W, np.prod((nodes - c[:, None, :]) ** al, axis=2))
        rhs = np.zeros((rwg.n, 3))
        for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
            pts = quad.points(rwg.verts[rwg.tris[side]])
            a = rwg.area[side]
            f = sgn * (rwg.length / (2 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
            t = np.cross(f, nrm[side][:, None, :])
            dlt = pts - c[:, None, :]
            g = np.zeros(pts.shape)
            for e in range(3):
                if al[e]:
                    ae = al.copy()
                    ae[e] -= 1
                    g[..., e] = al[e] * np.prod(dlt ** ae, axis=2)
            rhs += np.einsum("np,npe->ne", a[:, None] * quad.WEIGHTS, np.cross(t, g))
        scale = np.abs(W).max() * grid.h ** max(sum(alpha), 1)
        assert np.abs(lhs - rhs).max() <= 1e-12 * scale


def test_cfie_aim_equals_mom_when_everything_is_near(sphere_cfie):
    rwg, ZC = sphere_cfie
    op = aim.build_operator(rwg, K, 0.1 * LAM, 2, 10 * LAM, cfie_alpha=0.6)
    x = random_current(rwg.n, nrhs=2, seed=5)
    y = aim.matvec_fft(op, x)
    assert np.linalg.norm(y - (ZC @ x.T).T) <= 1e-13 * np.linalg.norm(y)
    np.testing.assert_allclose(op.zmom_diag, np.diag(ZC), rtol=1e-14, atol=0)


def test_cfie_fft_equals_direct_sum_and_approximates_mom(sphere_cfie):
    """The combined-field product by FFT equals its direct-sum definition, and
    with the configured near zone it approximates the dense combined-field
    matrix to the AIM error level; the far entries of its grid part (both
    terms, and the MFIE term alone) approximate the MOM entries of separated
    pairs. A flipped curl-weight sign (planted in the oracle) fails both."""
    from oracle import mfie

    rwg, ZC = sphere_cfie
    op = aim.build_operator(rwg, K, 0.1 * LAM, 2, 0.3 * LAM, cfie_alpha=0.6)
    x = random_current(rwg.n, nrhs=1, seed=6)[0]
    y = aim.matvec_fft(op, x)
    assert np.linalg.norm(y - aim.matvec_direct(op, x)) <= 1e-12 * np.linalg.norm(y)
    ref = ZC @ x
    assert np.linalg.norm(y - ref) <= 0.02 * np.linalg.norm(ref)
    far = np.array([(i, j) for i in range(0, rwg.n, 5) for j in range(0, rwg.n, 7)
                    if np.linalg.norm(rwg.centre[i] - rwg.centre[j]) > 0.5 * LAM])
    zh_far = ETA0 * mfie.zh_entries(rwg, K, far[:, 0], far[:, 1])
    for W, ok in ((op.curl, True), (-op.curl, False)):
        zg = aim.zgrid_entries(K, op.grid, op.lam, op.anc, far[:, 0], far[:, 1], W, 0.0)
        err = np.abs(zg - zh_far).max() / np.abs(zh_far).max()
        assert (err < 0.1) == ok, err
