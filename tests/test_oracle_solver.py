"""Pins for GMRES, the Mie series and err_theta_theta."""

import math

import numpy as np
import pytest

from oracle import aim, excitation, farfield, gmres, mie
from oracle.constants import wavelength, wavenumber
from oracle.rwg import build_rwg
from workloads import plate_mesh

F = 0.3e9
K = wavenumber(F)
LAM = wavelength(F)


@pytest.fixture(scope="module")
def plate():
    m = plate_mesh(1.0, F)
    rwg = build_rwg(m.verts, m.tris)
    op = aim.build_operator(rwg, K, 0.1 * LAM, 2, 0.3 * LAM)
    return rwg, op


def _dense(op):
    eye = np.eye(op.n, dtype=complex)
    return aim.matvec_fft(op, eye).T  # columns A e_j


@pytest.mark.parametrize("restart", [100, 7])
def test_gmres_matches_lu(plate, restart):
    rwg, op = plate
    A = _dense(op)
    b = excitation.planewave_rhs(rwg, K, 0.4, 0.9, 1)
    x, st = gmres.gmres(lambda v: A @ v, b, op.zmom_diag, 1e-10, restart=restart)
    assert st["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    xl = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xl) <= 1e-7 * np.linalg.norm(xl)


def test_gmres_zero_rhs(plate):
    rwg, op = plate
    x, st = gmres.gmres(lambda v: aim.matvec_fft(op, v), np.zeros(op.n, complex), op.zmom_diag, 1e-6)
    assert st["iters"] == 0 and np.all(x == 0)


def test_gmres_diag_is_mom_diagonal(plate):
    rwg, op = plate
    A = _dense(op)
    np.testing.assert_allclose(np.diag(A), op.zmom_diag, rtol=1e-12)


def test_mie_optical_theorem():
    for x in (0.3, 2.0, 16.0, 50.3):
        qext, qsca = mie.efficiencies(x)
        assert qext == pytest.approx(qsca, rel=1e-10)


def test_mie_limits():
    a = 1.0
    # Rayleigh: sigma_back = 9 pi a^2 (ka)^4
    k = 0.005
    s = mie.sigma_tt(k, a, np.array([0.0]), np.array([0.0]))[0, 0]
    assert s == pytest.approx(9 * math.pi * a**2 * (k * a) ** 4, rel=1e-4)
    # optics: sigma_back -> pi a^2
    k = 400.0
    s = mie.sigma_tt(k, a, np.array([0.0]), np.array([0.0]))[0, 0]
    assert s == pytest.approx(math.pi * a**2, rel=0.02)


def test_mie_scattering_integral():
    """Integrating |S1|^2 + |S2|^2 over angle gives Q_sca from the coefficients."""
    x = 4.0
    Th, w = np.polynomial.legendre.leggauss(200)
    Theta = np.arccos(Th)
    S1, S2 = mie.amplitudes(x, Theta)
    qsca_int = (1.0 / x**2) * np.sum(w * (np.abs(S1) ** 2 + np.abs(S2) ** 2))
    assert qsca_int == pytest.approx(mie.efficiencies(x)[1], rel=1e-10)


def test_err_tt_definition():
    th, ph = farfield.rcs_grid(5.0)
    rng = np.random.default_rng(0)
    s = rng.random((th.size, ph.size)) + 0.1
    assert farfield.err_tt(s, s, th) == 0.0
    assert farfield.err_tt(2 * s, s, th) == pytest.approx(1.0, rel=1e-14)
    t = s.copy()
    t[0, :] += 5.0  # theta = 0 row has zero weight
    assert farfield.err_tt(t, s, th) == 0.0
