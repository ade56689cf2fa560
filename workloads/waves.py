"""Plane-wave incidence sets.

A wave is ``(theta_inc, phi_inc, pol)``: it arrives from direction
r_hat(theta_inc, phi_inc), so it propagates along -r_hat, with unit amplitude
and polarisation theta_hat (pol=0) or phi_hat (pol=1) at (theta_inc, phi_inc).
The paper's case, an x-polarised wave travelling toward -z (Section 2.1), is
``(0, 0, 0)``.
"""

from __future__ import annotations

import math

import numpy as np


def normal_incidence() -> np.ndarray:
    """The x-polarised wave propagating toward -z."""
    return np.array([(0.0, 0.0, 0)], dtype=[("theta", "f8"), ("phi", "f8"), ("pol", "i4")])


def planewave_set(n_theta: int = 8) -> np.ndarray:
    """n_theta incidence angles theta_i = i*pi/(n_theta-1), phi = 0, each with
    theta_hat and phi_hat polarisation (2*n_theta waves, theta-major)."""
    out = []
    for i in range(n_theta):
        th = i * math.pi / (n_theta - 1) if n_theta > 1 else 0.0
        for pol in (0, 1):
            out.append((th, 0.0, pol))
    return np.array(out, dtype=[("theta", "f8"), ("phi", "f8"), ("pol", "i4")])
