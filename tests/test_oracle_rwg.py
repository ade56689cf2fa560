"""Pins for the RWG table: unknown counts, orientation and error paths."""

import os

import numpy as np
import pytest

from oracle import quadrature as quad
from oracle.rwg import MeshError, basis_on_points, build_rwg
from workloads import plate_mesh, sphere_mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_plate_unknowns.txt")


def _table1():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            L, N, chk = line.split()
            rows.append((float(L), int(N), chk == "1"))
    return rows


@pytest.mark.parametrize("L,N,check", [r for r in _table1() if r[0] <= 32])
def test_plate_unknowns_match_table1(L, N, check):
    """Plates meshed at 10 squares/lambda give Table 1's unknown counts."""
    m = plate_mesh(L, 0.3e9, squares_per_lambda=10)
    rwg = build_rwg(m.verts, m.tris)
    n = int(round(10 * L))
    assert rwg.n == 3 * n * n - 2 * n
    if check:
        assert rwg.n == N


def test_table1_large_rows_follow_structured_count():
    for L, N, check in _table1():
        n = int(round(10 * L))
        if check:
            assert 3 * n * n - 2 * n == N


@pytest.mark.parametrize("nf", [1, 2, 5])
def test_sphere_closed(nf):
    m = sphere_mesh(1.0, 0.3e9, nf=nf)
    rwg = build_rwg(m.verts, m.tris)
    assert m.nt == 20 * nf * nf
    assert rwg.n == 30 * nf * nf  # every edge interior
    assert m.nv - rwg.n + m.nt == 2  # Euler characteristic of a sphere
    # outward orientation: normals point away from the centre
    v = m.verts[m.tris]
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    assert np.all(np.einsum("tc,tc->t", nrm, v.mean(axis=1)) > 0)


def test_ordering_and_sides():
    m = plate_mesh(1.0, 0.3e9)
    rwg = build_rwg(m.verts, m.tris)
    e = rwg.edge
    assert np.all(e[:, 0] < e[:, 1])
    key = e[:, 0] * (m.nv + 1) + e[:, 1]
    assert np.all(np.diff(key) > 0)
    assert np.all(rwg.tplus < rwg.tminus)


def test_normal_current_continuity():
    """The normal component of f_n across its edge is 1 from both sides."""
    m = sphere_mesh(1.0, 0.3e9, nf=3)
    rwg = build_rwg(m.verts, m.tris)
    for n in range(0, rwg.n, 17):
        a, b = m.verts[rwg.edge[n]]
        mid = 0.5 * (a + b)
        # in-plane unit normal to the edge on each triangle, pointing T+ -> T-
        vals = []
        for t, free in ((rwg.tplus[n], rwg.vplus[n]), (rwg.tminus[n], rwg.vminus[n])):
            F, _ = basis_on_points(rwg, n, t, mid[None, :])
            tv = m.verts[m.tris[t]]
            nt = np.cross(tv[1] - tv[0], tv[2] - tv[0])
            u = np.cross(b - a, nt)
            u /= np.linalg.norm(u)
            if np.dot(u, mid - m.verts[rwg.vplus[n]]) < 0 and t == rwg.tplus[n]:
                u = -u
            if np.dot(u, m.verts[rwg.vminus[n]] - mid) < 0 and t == rwg.tminus[n]:
                u = -u
            vals.append(float(np.dot(F[0], u)))
        assert vals[0] == pytest.approx(1.0, rel=1e-12)
        assert vals[1] == pytest.approx(1.0, rel=1e-12)


def test_divergence_integrates_to_zero():
    m = plate_mesh(1.0, 0.3e9)
    rwg = build_rwg(m.verts, m.tris)
    tot = rwg.length / rwg.area[rwg.tplus] * rwg.area[rwg.tplus] - rwg.length / rwg.area[rwg.tminus] * rwg.area[rwg.tminus]
    assert np.max(np.abs(tot)) < 1e-15 * rwg.length.max()
    assert quad.WEIGHTS.sum() == pytest.approx(1.0)


def test_mesh_errors():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=float)
    with pytest.raises(MeshError):  # edge (0,1) shared by three triangles
        build_rwg(v, np.array([[0, 1, 2], [0, 1, 3], [1, 0, 4]]))
    with pytest.raises(MeshError):
        build_rwg(v, np.array([[0, 1, 7]]))
    with pytest.raises(MeshError):
        build_rwg(np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], dtype=float), np.array([[0, 1, 2]]))
