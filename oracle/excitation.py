"""Plane-wave excitation vector (tested incident field).

Test infrastructure only. The plate and sphere are lit by an x-polarised
plane wave travelling toward -z (Section 2.1). A wave arriving from
r_hat(theta_i, phi_i) has direction k_hat = -r_hat and field

    E_inc(r) = p_hat exp(-j k k_hat . r),  p_hat = theta_hat or phi_hat,

and the Galerkin right-hand side is V_m = int f_m . E_inc dS, evaluated with
the 7-point rule on T+ and T-.
"""

from __future__ import annotations

import math

import numpy as np

from . import quadrature as quad
from .rwg import RWG


def unit_vectors(theta: float, phi: float):
    st, ct, sp, cp = math.sin(theta), math.cos(theta), math.sin(phi), math.cos(phi)
    r_hat = np.array([st * cp, st * sp, ct])
    th_hat = np.array([ct * cp, ct * sp, -st])
    ph_hat = np.array([-sp, cp, 0.0])
    return r_hat, th_hat, ph_hat


def planewave_rhs(rwg: RWG, k: float, theta: float, phi: float, pol: int) -> np.ndarray:
    r_hat, th_hat, ph_hat = unit_vectors(theta, phi)
    k_hat = -r_hat
    p_hat = th_hat if pol == 0 else ph_hat
    V = np.zeros(rwg.n, dtype=np.complex128)
    for side, free, sgn in ((rwg.tplus, rwg.vplus, 1.0), (rwg.tminus, rwg.vminus, -1.0)):
        tri = rwg.verts[rwg.tris[side]]  # (N, 3, 3)
        pts = quad.points(tri)  # (N, 7, 3)
        a = rwg.area[side]
        f = sgn * (rwg.length / (2.0 * a))[:, None, None] * (pts - rwg.verts[free][:, None, :])
        e = np.exp(-1j * k * (pts @ k_hat))  # (N, 7)
        V += a * np.einsum("p,np,np->n", quad.WEIGHTS, f @ p_hat, e)
    return V
