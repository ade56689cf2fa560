"""Scattered far field, bistatic RCS and the err_theta_theta measure.

Test infrastructure only.

Far field: with the current J = sum_n I_n f_n and time convention exp(+jwt),
the radiation vector is N(r_hat) = int J(r') exp(+j k r_hat . r') dS' and the
far scattered field is E = -j k eta exp(-jkr)/(4 pi r) [N - (r_hat . N) r_hat].
For a unit-amplitude incident wave the bistatic RCS is

    sigma_tt(theta, phi) = (k eta)^2 / (4 pi) |theta_hat . N|^2   (m^2).

err_theta_theta is eq. (1) of the paper (Section 2.2): the relative
root-mean-square difference of sigma_tt over the sphere of directions,
weighted by sin(theta). We evaluate it as the discrete sum over a regular
(theta, phi) grid with sin(theta) weights.
"""

from __future__ import annotations

import math

import numpy as np

from . import quadrature as quad
from .constants import ETA0
from .rwg import RWG


def rcs_grid(step_deg: float = 1.0):
    theta = np.deg2rad(np.arange(0.0, 180.0 + 1e-9, step_deg))
    phi = np.deg2rad(np.arange(0.0, 360.0 - 1e-9, step_deg))
    return theta, phi


def radiation_vector(rwg: RWG, k: float, I: np.ndarray, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """N(r_hat) on the (theta, phi) grid: (ntheta, nphi, 3) complex."""
    # current density at each triangle quadrature point, times A * w
    pts_all = []
    J_all = []
    for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
        tri = rwg.verts[rwg.tris[side]]
        pts = quad.points(tri)  # (N, 7, 3)
        a = rwg.area[side]
        f = sgn * (rwg.length / (2.0 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
        J = (I * a)[:, None, None] * quad.WEIGHTS[None, :, None] * f
        pts_all.append(pts.reshape(-1, 3))
        J_all.append(J.reshape(-1, 3))
    P = np.concatenate(pts_all)
    J = np.concatenate(J_all)
    th, ph = np.meshgrid(theta, phi, indexing="ij")
    rh = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=-1).reshape(-1, 3)
    out = np.zeros((rh.shape[0], 3), dtype=np.complex128)
    chunk = max(1, 4_000_000 // max(1, P.shape[0]))
    for s in range(0, rh.shape[0], chunk):
        ph_ = np.exp(1j * k * (rh[s:s + chunk] @ P.T))  # (c, P)
        out[s:s + chunk] = ph_ @ J
    return out.reshape(th.shape + (3,))


def sigma_tt(rwg: RWG, k: float, I: np.ndarray, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    Nv = radiation_vector(rwg, k, I, theta, phi)
    th, ph = np.meshgrid(theta, phi, indexing="ij")
    th_hat = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=-1)
    Nt = np.einsum("tpc,tpc->tp", Nv, th_hat)
    return (k * ETA0) ** 2 / (4 * math.pi) * np.abs(Nt) ** 2


def err_tt(sigma: np.ndarray, sigma_ref: np.ndarray, theta: np.ndarray) -> float:
    """Eq. (1): relative RMS error of sigma_tt, sin(theta)-weighted."""
    w = np.sin(theta)[:, None]
    num = np.sum(w * np.abs(sigma - sigma_ref) ** 2)
    den = np.sum(w * np.abs(sigma_ref) ** 2)
    return float(np.sqrt(num / den))
