"""RWG (Rao-Wilton-Glisson 1982) basis functions on a triangle mesh.

Test infrastructure only. The paper's scatterers are PEC surfaces meshed
with triangles (Section 2.1) and discretised with the method of moments; its
unknowns are RWG edge currents. Conventions (the paper is silent on them):

* one unknown per interior edge (an edge shared by exactly two triangles);
  boundary edges of an open surface carry none; an edge shared by three or
  more triangles is an error;
* unknowns are ordered by (min vertex id, max vertex id) of their edge;
* T+ is the adjacent triangle with the smaller index, T- the other;
* f_n(r) = (l_n / 2A+)(r - p+) on T+ and (l_n / 2A-)(p- - r) on T-, with
  p+- the vertex of T+- opposite the edge, so div f_n = +l_n/A+ on T+ and
  -l_n/A- on T-;
* the centre of basis n is the mean of the centroids of T+ and T-.
"""

from __future__ import annotations

import dataclasses

import numpy as np


class MeshError(ValueError):
    pass


@dataclasses.dataclass
class RWG:
    verts: np.ndarray  # (nv, 3)
    tris: np.ndarray  # (nt, 3)
    edge: np.ndarray  # (N, 2) vertex ids, sorted
    tplus: np.ndarray  # (N,)
    tminus: np.ndarray  # (N,)
    vplus: np.ndarray  # (N,) free vertex id of T+
    vminus: np.ndarray  # (N,) free vertex id of T-
    length: np.ndarray  # (N,)
    area: np.ndarray  # (nt,)
    centroid: np.ndarray  # (nt, 3)
    centre: np.ndarray  # (N, 3)
    # per triangle, per local vertex i: basis whose free vertex is local vertex
    # i (-1 if that edge carries no unknown) and its sign (+1 on T+, -1 on T-)
    tri_basis: np.ndarray  # (nt, 3)
    tri_sign: np.ndarray  # (nt, 3)

    @property
    def n(self) -> int:
        return int(self.edge.shape[0])


def triangle_areas(verts, tris):
    v = verts[tris]
    return 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)


def build_rwg(verts: np.ndarray, tris: np.ndarray, min_area: float = 0.0) -> RWG:
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    nv = verts.shape[0]
    nt = tris.shape[0]
    if nv <= 0 or nt <= 0:
        raise MeshError("empty mesh")
    if tris.min() < 0 or tris.max() >= nv:
        raise MeshError("vertex index out of range")
    if np.any(tris[:, 0] == tris[:, 1]) or np.any(tris[:, 1] == tris[:, 2]) or np.any(tris[:, 0] == tris[:, 2]):
        raise MeshError("triangle with repeated vertex")
    area = triangle_areas(verts, tris)
    if np.any(area <= min_area):
        raise MeshError("degenerate triangle")

    # every triangle edge, keyed by its sorted vertex pair; the edge opposite
    # local vertex i joins the other two vertices
    rows = []
    for i in range(3):
        a = tris[:, (i + 1) % 3]
        b = tris[:, (i + 2) % 3]
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        rows.append(np.stack([lo, hi, np.arange(nt), np.full(nt, i)], axis=1))
    e = np.concatenate(rows)
    order = np.lexsort((e[:, 2], e[:, 1], e[:, 0]))  # by (lo, hi, triangle)
    e = e[order]
    key_change = np.ones(e.shape[0], dtype=bool)
    key_change[1:] = (e[1:, 0] != e[:-1, 0]) | (e[1:, 1] != e[:-1, 1])
    starts = np.flatnonzero(key_change)
    counts = np.diff(np.append(starts, e.shape[0]))
    if np.any(counts > 2):
        raise MeshError("edge shared by more than two triangles")
    inner = starts[counts == 2]
    first = e[inner]  # smaller triangle index (lexsorted) -> T+
    second = e[inner + 1]
    N = inner.shape[0]
    edge = first[:, :2].copy()
    tplus = first[:, 2].copy()
    tminus = second[:, 2].copy()
    vplus = tris[tplus, first[:, 3]]
    vminus = tris[tminus, second[:, 3]]
    length = np.linalg.norm(verts[edge[:, 0]] - verts[edge[:, 1]], axis=1)
    centroid = verts[tris].sum(axis=1) / 3.0
    centre = 0.5 * (centroid[tplus] + centroid[tminus])
    tri_basis = np.full((nt, 3), -1, dtype=np.int64)
    tri_sign = np.zeros((nt, 3), dtype=np.int64)
    n_ids = np.arange(N)
    tri_basis[tplus, first[:, 3]] = n_ids
    tri_sign[tplus, first[:, 3]] = 1
    tri_basis[tminus, second[:, 3]] = n_ids
    tri_sign[tminus, second[:, 3]] = -1
    return RWG(verts=verts, tris=tris, edge=edge, tplus=tplus, tminus=tminus,
               vplus=vplus, vminus=vminus, length=length, area=area,
               centroid=centroid, centre=centre, tri_basis=tri_basis,
               tri_sign=tri_sign)


def basis_on_points(rwg: RWG, n: int, tri: int, pts: np.ndarray):
    """f_n and div f_n at points of triangle ``tri`` (which must be T+ or T-
    of basis n). Returns (F (P,3), div scalar)."""
    if tri == rwg.tplus[n]:
        s, p = 1.0, rwg.verts[rwg.vplus[n]]
    elif tri == rwg.tminus[n]:
        s, p = -1.0, rwg.verts[rwg.vminus[n]]
    else:
        raise ValueError("triangle does not support basis")
    a = rwg.area[tri]
    l = rwg.length[n]
    return s * (l / (2.0 * a)) * (pts - p), s * l / a
