"""Pins for the closed-form triangle potentials against Duffy quadrature.

The closed forms (Wilton et al. 1984; Graglia 1993) are checked against an
independent route: the triangle is split into (signed) sub-triangles with
apex at the projection of the observation point, each mapped to the unit
square with the Duffy transform r' = rho + u[(a - rho) + v (b - a)], whose
Jacobian u cancels the 1/R singularity; the result is integrated with
composite Gauss-Legendre rules (geometrically graded in u).
"""

import numpy as np
import pytest

from oracle.potentials import triangle_potentials


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _composite(edges, npts=24):
    us, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        x, w = _gl(npts, a, b)
        us.append(x)
        ws.append(w)
    return np.concatenate(us), np.concatenate(ws)


def _u_rule():
    return _composite(np.concatenate([[0.0], np.logspace(-9, 0, 19)]))


def _v_rule():
    g = np.logspace(-8, np.log10(0.5), 16)
    return _composite(np.unique(np.concatenate([[0.0, 1.0], g, 1.0 - g, np.linspace(0, 1, 9)])))


def duffy(tri, r):
    v0, v1, v2 = tri
    n = np.cross(v1 - v0, v2 - v0)
    n /= np.linalg.norm(n)
    d = np.dot(r - v0, n)
    rho = r - d * n
    u, wu = _u_rule()
    v, wv = _v_rule()
    I1 = 0.0
    Iv = np.zeros(3)
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        cr = np.cross(a - rho, b - rho)
        jac = np.dot(cr, n)  # signed, = 2 * signed area
        U, Vv = np.meshgrid(u, v, indexing="ij")
        W = np.outer(wu, wv)
        pts = rho + U[..., None] * ((a - rho) + Vv[..., None] * (b - a))
        diff = pts - r
        R = np.linalg.norm(diff, axis=-1)
        I1 += np.sum(W * U * jac / R)
        Iv += np.einsum("uv,uvc->c", W * U * jac / R, diff)
    return I1, Iv


TRI = np.array([[0.1, -0.2, 0.05], [1.3, 0.1, -0.1], [0.2, 0.9, 0.3]])


def _frame():
    v0, v1, v2 = TRI
    n = np.cross(v1 - v0, v2 - v0)
    n /= np.linalg.norm(n)
    return n


@pytest.mark.parametrize("bary,height", [
    ((1 / 3, 1 / 3, 1 / 3), 0.0),      # centroid, in plane
    ((0.7, 0.2, 0.1), 0.0),            # interior, in plane
    ((0.05, 0.05, 0.9), 0.0),          # near a vertex
    ((1.4, -0.3, -0.1), 0.0),          # outside, in plane
    ((0.3, 0.3, 0.4), 0.25),           # above
    ((0.3, 0.3, 0.4), -0.02),          # just below
    ((-0.5, 0.8, 0.7), 0.4),           # above, outside
])
def test_closed_form_matches_duffy(bary, height):
    r = np.asarray(bary) @ TRI + height * _frame()
    I1, Iv = triangle_potentials(TRI, r[None, :])
    J1, Jv = duffy(TRI, r)
    assert I1[0] == pytest.approx(J1, rel=1e-11)
    np.testing.assert_allclose(Iv[0], Jv, rtol=1e-10, atol=1e-11 * np.linalg.norm(Jv))


def test_far_point_limit():
    # far away, 1/R -> area / distance
    far = np.array([40.0, -25.0, 70.0])
    I1, Iv = triangle_potentials(TRI, far[None, :])
    v0, v1, v2 = TRI
    area = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    c = TRI.mean(axis=0)
    assert I1[0] == pytest.approx(area / np.linalg.norm(far - c), rel=1e-4)
    np.testing.assert_allclose(Iv[0], area * (c - far) / np.linalg.norm(far - c), rtol=1e-3)
