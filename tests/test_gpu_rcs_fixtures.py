"""Solve-level parity at the benchmark sizes: the GPU's converged solves
(mixed and FP64 paths, tolerance 1e-4 on the FP64 residual, Section 2.2)
against the FP64 oracle's solves (tolerance 1e-6), through the RCS error
measure err_theta_theta of eq. (1) on the 2-degree grid. The oracle's
sigma_theta_theta is stored under tests/golden/ by make_rcs_fixtures.py,
which calls only the oracle. Bar: err_theta_theta(GPU, oracle) <= 1e-3."""

import os
import sys

import numpy as np
import pytest

from oracle import farfield as off

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_rcs_fixtures as fx  # noqa: E402

ERR_BAR = 1e-3


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fixtures(case):
    out = []
    for i in range(len(fx.CASES[case][2])):
        path = fx.fixture_path(case, i)
        if not os.path.exists(path):
            pytest.fail(f"missing oracle fixture {path} (run tests/golden/make_rcs_fixtures.py {case})")
        out.append(fx.load_fixture(path))
    return out


def _check_meta(meta, mesh, n):
    assert int(meta["n"]) == n
    assert float(meta["freq_hz"]) == mesh.freq_hz
    assert float(meta["oracle_residual"]) <= float(meta["oracle_tol"])


@pytest.mark.parametrize("case", ["plate16", "sphere8"])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_single_scatterer_solve_matches_oracle_rcs(case, prec):
    from paper_1010_1456_amd import aim as A

    (sig_ref, meta), = _fixtures(case)
    recipe, alpha, waves, _, _ = fx.CASES[case]
    mesh = fx._mesh(recipe)
    _log(f"[rcs {case} {prec}] set-up")
    plan = A.Plan([(mesh.verts, mesh.tris, mesh.freq_hz)], cfie_alpha=alpha)
    _check_meta(meta, mesh, plan.n_total)
    P = A.AIM_MIXED if prec == "mixed" else A.AIM_FP64
    _log(f"[rcs {case} {prec}] solve")
    x, st = plan.solve(waves, P, tol=1e-4, max_iter=6000)
    assert st[0]["converged"] and st[0]["residual"] <= 1e-4
    th, ph = off.rcs_grid(2.0)
    sig = plan.rcs(x, th, ph)[0, 0]
    err = off.err_tt(sig, sig_ref, th)
    _log(f"[rcs {case} {prec}] its={st[0]['iterations']} residual={st[0]['residual']:.2e} "
         f"err_tt={err:.2e}")
    assert err <= ERR_BAR
    plan.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_members_oblique_waves_match_oracle_rcs(prec):
    """Two members of the uneven batch (the jittered 4-lambda plate, EFIE, and
    2-lambda sphere, CFIE alpha = 0.6) in one plan, lit by two oblique waves:
    every (scatterer, wave) system converges and its RCS matches the
    oracle's."""
    from paper_1010_1456_amd import aim as A

    refs = {c: _fixtures(c) for c in ("b6plate4", "b6sphere2")}
    meshes = [fx._mesh(fx.CASES[c][0]) for c in ("b6plate4", "b6sphere2")]
    waves = fx.OBLIQUE
    assert fx.CASES["b6plate4"][2] == waves and fx.CASES["b6sphere2"][2] == waves
    _log(f"[rcs batch {prec}] set-up")
    plan = A.Plan([(m.verts, m.tris, m.freq_hz) for m in meshes], cfie_alpha=0.6,
                  cfie_closed_only=True)
    inf = plan.info()
    assert inf["cfie_alpha"] == [None, 0.6]
    P = A.AIM_MIXED if prec == "mixed" else A.AIM_FP64
    _log(f"[rcs batch {prec}] solve")
    x, st = plan.solve(waves, P, tol=1e-4, max_iter=6000)
    assert len(st) == 2 * len(waves)
    th, ph = off.rcs_grid(2.0)
    sig = plan.rcs(x, th, ph)  # (mesh, wave, theta, phi)
    for mi, case in enumerate(("b6plate4", "b6sphere2")):
        for wi in range(len(waves)):
            q = st[mi * len(waves) + wi]
            assert (q["mesh"], q["wave"]) == (mi, wi)
            assert q["converged"] and q["residual"] <= 1e-4, q
            sig_ref, meta = refs[case][wi]
            _check_meta(meta, meshes[mi], inf["n"][mi])
            err = off.err_tt(sig[mi, wi], sig_ref, th)
            _log(f"[rcs batch {prec}] {case} wave {wi}: its={q['iterations']} err_tt={err:.2e}")
            assert err <= ERR_BAR
    plan.close()
