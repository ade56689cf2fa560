"""GPU parity of the combined-field (CFIE) path against the FP64 oracle.

Bars as for the EFIE: curl weights, near-zone matrix and preconditioner
diagonal to 1e-12-1e-13 of their largest entry; right-hand sides to 1e-13;
product FP64 <= 1e-10, mixed <= 2e-5; solved currents err_theta_theta <= 1e-3
against the oracle's solution, and the sphere against the Mie series.
"""

import sys

import numpy as np
import pytest

from oracle import aim as oaim
from oracle import farfield as off
from oracle import gmres as ogmres
from oracle import mfie as omfie
from oracle import mie as omie
from oracle.constants import wavenumber
from oracle.rwg import build_rwg
from workloads import planewave_set, random_current, sphere_mesh

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# name -> (radius in wavelengths, nf, stencil order M, alpha)
CASES = {
    "sphere05": (0.5, 4, 2, 0.6),
    "sphere05_m3": (0.5, 4, 3, 0.6),
    "sphere05_mfie": (0.5, 4, 2, 0.0),
}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Case:
    def __init__(self, name):
        from paper_1010_1456_amd import aim as A

        radius, nf, M, alpha = CASES[name]
        self.alpha = alpha
        self.radius = radius
        self.mesh = m = sphere_mesh(radius, 0.3e9, nf=nf)
        self.k = wavenumber(m.freq_hz)
        _log(f"[cfie case {name}] oracle set-up (M={M}, alpha={alpha})")
        self.rwg = build_rwg(m.verts, m.tris)
        self.op = oaim.build_operator(self.rwg, self.k, 0.1 * m.lam, M, 0.3 * m.lam, cfie_alpha=alpha)
        _log(f"[cfie case {name}] GPU set-up N={self.rwg.n}")
        self.plan = A.Plan([(m.verts, m.tris, m.freq_hz)], order=M, cfie_alpha=alpha)
        torch.cuda.synchronize()


_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = Case(name)
    return _cache[name]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("name", list(CASES))
def test_operator_data(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    assert c.plan.info()["cfie_alpha"] == [c.alpha]
    W = c.plan.export(0, A.AIM_DATA_CURL64)
    assert np.abs(W - c.op.curl).max() <= 1e-13 * np.abs(c.op.curl).max()
    near = c.plan.export(0, A.AIM_DATA_NEAR64)
    ref = c.op.near.data
    assert np.abs(near - ref).max() <= 1e-12 * np.abs(ref).max()
    zd = c.plan.export(0, A.AIM_DATA_ZDIAG64)
    assert np.abs(zd - c.op.zmom_diag).max() <= 1e-12 * np.abs(c.op.zmom_diag).max()


@pytest.mark.parametrize("name", ["sphere05", "sphere05_mfie"])
def test_excitation(name):
    c = case(name)
    waves = planewave_set(4)
    b = c.plan.excitation([tuple(w) for w in waves]).cpu().numpy()
    for i, w in enumerate(waves):
        ref = omfie.planewave_rhs_c(c.rwg, c.k, float(w["theta"]), float(w["phi"]), int(w["pol"]),
                                    c.alpha)
        assert np.linalg.norm(b[i] - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", list(CASES))
def test_matvec(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    x = random_current(c.rwg.n, nrhs=4, seed=21)
    ref = oaim.matvec_fft(c.op, x)
    y = c.plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    for r in range(4):
        assert rel(y[r], ref[r]) <= 1e-10
    x32 = x.astype(np.complex64)
    y32 = c.plan.matvec(torch.from_numpy(x32).cuda(), A.AIM_MIXED).cpu().numpy()
    ref32 = oaim.matvec_fft(c.op, x32.astype(np.complex128))
    for r in range(4):
        assert rel(y32[r].astype(np.complex128), ref32[r]) <= 2e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_matches_oracle_and_mie(prec):
    """CFIE (alpha 0.6) solve of the 0.5-lambda sphere, tol 1e-6: RCS against
    the oracle's own solution (<= 1e-3) and against the Mie series."""
    from paper_1010_1456_amd import aim as A

    c = case("sphere05")
    wave = (0.0, 0.0, 0)
    b = omfie.planewave_rhs_c(c.rwg, c.k, *wave, c.alpha)
    xo, st_o = ogmres.gmres(lambda v: oaim.matvec_fft(c.op, v), b, c.op.zmom_diag, 1e-10)
    assert st_o["converged"]
    P = A.AIM_FP64 if prec == "fp64" else A.AIM_MIXED
    x, st = c.plan.solve([wave], P, tol=1e-6)
    assert st[0]["converged"] and st[0]["residual"] <= 1e-6
    xn = x.cpu().numpy()[0]
    res = np.linalg.norm(b - oaim.matvec_fft(c.op, xn)) / np.linalg.norm(b)
    assert res <= 1.05e-6
    th, ph = off.rcs_grid(2.0)
    sg = c.plan.rcs(x, th, ph)[0, 0]
    so = off.sigma_tt(c.rwg, c.k, xo, th, ph)
    err = off.err_tt(sg, so, th)
    sm = omie.sigma_tt(c.k, c.radius * c.mesh.lam, th, ph)
    err_mie = off.err_tt(sg, sm, th)
    _log(f"[cfie solve {prec}] its={st[0]['iterations']} err_tt vs oracle {err:.2e}, vs Mie {err_mie:.3f}")
    assert err <= 1e-3
    assert err_mie < 0.06


def test_cfie_converges_faster_than_efie_on_a_larger_sphere():
    """A 2-lambda-radius sphere (the batch's largest closed member size class):
    the combined field converges in far fewer iterations than the EFIE and
    agrees with the Mie series at least as well."""
    from paper_1010_1456_amd import aim as A

    mesh = sphere_mesh(2.0, 0.3e9)
    k = wavenumber(mesh.freq_hz)
    th, ph = off.rcs_grid(2.0)
    sm = omie.sigma_tt(k, 2.0 * mesh.lam, th, ph)
    out = {}
    for alpha in (None, 0.6):
        plan = A.Plan([(mesh.verts, mesh.tris, mesh.freq_hz)], cfie_alpha=alpha)
        x, st = plan.solve([(0.0, 0.0, 0)], A.AIM_MIXED, tol=1e-4, max_iter=2000)
        out[alpha] = (st[0]["iterations"], off.err_tt(plan.rcs(x, th, ph)[0, 0], sm, th), st[0]["converged"])
        plan.close()
    _log(f"[cfie vs efie, 2-lambda sphere] EFIE its/err {out[None][:2]}, CFIE its/err {out[0.6][:2]}")
    assert out[0.6][2] and out[0.6][0] < out[None][0]


def test_batch_with_the_papers_formulations():
    """A plate and a sphere in one plan with the combined field on closed
    meshes only: the plate takes the EFIE, the sphere the CFIE, and the
    batched product and solve equal those of the single-mesh plans."""
    from paper_1010_1456_amd import aim as A
    from workloads import plate_mesh

    plate = plate_mesh(2.0, 0.3e9, jitter_seed=1001)
    sph = sphere_mesh(0.5, 0.3e9, nf=4)
    batch = A.Plan([(m.verts, m.tris, m.freq_hz) for m in (plate, sph)], cfie_alpha=0.6,
                   cfie_closed_only=True)
    inf = batch.info()
    assert inf["cfie_alpha"] == [None, 0.6]
    singles = [A.Plan([(plate.verts, plate.tris, plate.freq_hz)]),
               A.Plan([(sph.verts, sph.tris, sph.freq_hz)], cfie_alpha=0.6)]
    x = random_current(inf["n_total"], nrhs=2, seed=31)
    y = batch.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    waves = [(0.0, 0.0, 0), (0.7, 0.3, 1)]
    xb, stb = batch.solve(waves, A.AIM_MIXED, tol=1e-6)
    xb = xb.cpu().numpy()
    for i, pl in enumerate(singles):
        lo, n = inf["offset"][i], inf["n"][i]
        ys = pl.matvec(torch.from_numpy(np.ascontiguousarray(x[:, lo:lo + n])).cuda(), A.AIM_FP64).cpu().numpy()
        assert rel(y[:, lo:lo + n], ys) <= 1e-13
        xs, sts = pl.solve(waves, A.AIM_MIXED, tol=1e-6)
        assert rel(xb[:, lo:lo + n], xs.cpu().numpy()) <= 1e-5
        pl.close()
    batch.close()


def _cube_mesh(side_lambda, freq_hz, n):
    """Closed cube, n x n squares per face, faces on the grid planes of an
    h = side / (6 n / 6) grid when side = n h; outward normals."""
    lam = 299_792_458.0 / freq_hz
    index, verts, tris = {}, [], []

    def vid(p):
        if p not in index:
            index[p] = len(verts)
            verts.append(p)
        return index[p]

    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s in (0, n):
            for u in range(n):
                for v in range(n):
                    def pt(du, dv):
                        p = [0, 0, 0]
                        p[a], p[b], p[c] = s, u + du, v + dv
                        return vid(tuple(p))
                    q = [pt(0, 0), pt(1, 0), pt(1, 1), pt(0, 1)]
                    t1, t2 = (q[0], q[1], q[2]), (q[0], q[2], q[3])
                    if s == 0:  # e_b x e_c = +e_a points inward on this face
                        t1, t2 = t1[::-1], t2[::-1]
                    tris += [t1, t2]
    v = (np.asarray(verts, dtype=float) / n - 0.5) * side_lambda * lam
    return v, np.asarray(tris, dtype=np.int32)


def test_grid_aligned_cube():
    """A closed cube whose faces lie on grid planes: off a face the projection
    weights vanish while the curl weights do not, so those grid nodes must be
    propagated too. Combined-field products against the oracle."""
    from paper_1010_1456_amd import aim as A

    freq = 0.3e9
    verts, tris = _cube_mesh(0.6, freq, 6)
    k = wavenumber(freq)
    lam = 299_792_458.0 / freq
    rwg = build_rwg(verts, tris)
    op = oaim.build_operator(rwg, k, 0.1 * lam, 2, 0.3 * lam, cfie_alpha=0.6)
    assert tuple(int(v) for v in op.grid.n) == (7, 7, 7)
    zero_lam = (np.abs(op.lam).max(axis=1) == 0) & (np.abs(op.curl).max(axis=1) > 0)
    assert zero_lam.any()  # nodes reached by curl weights only
    plan = A.Plan([(verts, tris, freq)], cfie_alpha=0.6)
    x = random_current(rwg.n, nrhs=2, seed=41)
    ref = oaim.matvec_fft(op, x)
    y = plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    for r in range(2):
        assert rel(y[r], ref[r]) <= 1e-10
    x32 = x.astype(np.complex64)
    y32 = plan.matvec(torch.from_numpy(x32).cuda(), A.AIM_MIXED).cpu().numpy()
    ref32 = oaim.matvec_fft(op, x32.astype(np.complex128))
    for r in range(2):
        assert rel(y32[r].astype(np.complex128), ref32[r]) <= 2e-5
    plan.close()
