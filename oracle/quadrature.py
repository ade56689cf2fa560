"""Seven-point degree-5 triangle rule (Radon's rule; Stroud 1971, T2:5-1).

Test infrastructure only. The configured surface quadrature is a 7-point
rule; we read it as Radon's degree-5 rule, exact for all polynomials of total
degree <= 5 over a triangle. Points are barycentric (l0, l1, l2); weights sum
to one and are multiplied by the triangle area.
"""

import math

import numpy as np

_S15 = math.sqrt(15.0)
_A = (6.0 - _S15) / 21.0
_B = (6.0 + _S15) / 21.0
_WA = (155.0 - _S15) / 1200.0
_WB = (155.0 + _S15) / 1200.0

BARY = np.array([
    [1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0],
    [1.0 - 2.0 * _A, _A, _A],
    [_A, 1.0 - 2.0 * _A, _A],
    [_A, _A, 1.0 - 2.0 * _A],
    [1.0 - 2.0 * _B, _B, _B],
    [_B, 1.0 - 2.0 * _B, _B],
    [_B, _B, 1.0 - 2.0 * _B],
])
WEIGHTS = np.array([9.0 / 40.0, _WA, _WA, _WA, _WB, _WB, _WB])


def points(tri_xyz: np.ndarray) -> np.ndarray:
    """Quadrature points of triangles. tri_xyz: (..., 3 vertices, 3) -> (..., 7, 3)."""
    return np.einsum("pv,...vc->...pc", BARY, tri_xyz)
