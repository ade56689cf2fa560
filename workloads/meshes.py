"""Triangulated PEC benchmark surfaces (paper Section 2.1).

The paper benchmarks a square plate centred at the origin in the x-y plane
and a sphere centred at the origin, both meshed at an average edge of about
lambda/9, with the size grown by doubling the frequency. These generators
build the same two families, in units of wavelengths scaled to metres:

* ``plate_mesh``: n x n structured squares per side, each split along its
  (i, j)-(i+1, j+1) diagonal, counter-clockwise about +z.
* ``sphere_mesh``: class-I geodesic sphere; every icosahedron face is split
  into nf^2 triangles and the vertices are projected radially onto radius a.
  Shared vertices are merged through integer barycentric keys, so the mesh is
  closed and consistently outward-oriented.

Optional seeded jitter (``jitter_seed``) moves every vertex by at most 2% of
the mean edge: plate interior vertices in x-y, plate boundary vertices along
their boundary side only, corners fixed; sphere vertices in 3-D followed by
renormalisation to radius a.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum, m/s


def wavelength(freq_hz: float) -> float:
    return C0 / float(freq_hz)


@dataclasses.dataclass
class Mesh:
    verts: np.ndarray  # (nv, 3) float64, metres
    tris: np.ndarray  # (nt, 3) int32, 0-based
    freq_hz: float
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.verts.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])

    @property
    def lam(self) -> float:
        return wavelength(self.freq_hz)


def _mean_edge(verts: np.ndarray, tris: np.ndarray) -> float:
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(verts[e[:, 0]] - verts[e[:, 1]], axis=1).mean())


def plate_mesh(side_lambda: float, freq_hz: float, squares_per_lambda: int = 9,
               jitter_seed: int | None = None, name: str = "") -> Mesh:
    """Square plate of side ``side_lambda`` wavelengths in the z=0 plane."""
    lam = wavelength(freq_hz)
    n = int(round(squares_per_lambda * side_lambda))
    if n < 1:
        raise ValueError("plate needs at least one square per side")
    s = np.arange(n + 1, dtype=np.float64) / n - 0.5  # in units of the side
    X, Y = np.meshgrid(s, s, indexing="xy")  # vertex (i, j) -> row j, column i
    vl = np.stack([X.ravel(), Y.ravel(), np.zeros((n + 1) ** 2)], axis=1) * side_lambda
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v00 = j * (n + 1) + i
    v10 = v00 + 1
    v11 = v00 + (n + 1) + 1
    v01 = v00 + (n + 1)
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    if jitter_seed is not None:
        ebar = _mean_edge(vl, tris)
        rng = np.random.default_rng(jitter_seed)
        ii = np.tile(np.arange(n + 1), n + 1)
        jj = np.repeat(np.arange(n + 1), n + 1)
        bx = (ii == 0) | (ii == n)
        by = (jj == 0) | (jj == n)
        interior = ~bx & ~by
        corner = bx & by
        side_x = by & ~bx  # on y=const boundary: slides along x
        side_y = bx & ~by  # on x=const boundary: slides along y
        d2 = rng.uniform(-1.0, 1.0, size=(vl.shape[0], 2))
        amp2 = 0.02 * ebar / math.sqrt(2.0)
        amp1 = 0.02 * ebar
        vl = vl.copy()
        vl[interior, 0] += amp2 * d2[interior, 0]
        vl[interior, 1] += amp2 * d2[interior, 1]
        vl[side_x, 0] += amp1 * d2[side_x, 0]
        vl[side_y, 1] += amp1 * d2[side_y, 1]
        assert not np.any(corner & interior)
    return Mesh(verts=vl * lam, tris=tris, freq_hz=float(freq_hz),
                name=name or f"plate{side_lambda:g}")


_PHI = (1.0 + math.sqrt(5.0)) / 2.0
_ICO_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
], dtype=np.float64)
_ICO_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
], dtype=np.int64)


def _geodesic_unit(nf: int):
    """Unit-radius class-I geodesic sphere with nf^2 triangles per face."""
    keymap: dict = {}
    pts = []

    def vid(face, i, j):
        a, b, c = (int(v) for v in _ICO_F[face])
        w = {a: nf - i - j}
        w[b] = w.get(b, 0) + i
        w[c] = w.get(c, 0) + j
        key = tuple(sorted((k, v) for k, v in w.items() if v != 0))
        idx = keymap.get(key)
        if idx is None:
            idx = len(pts)
            keymap[key] = idx
            p = (nf - i - j) * _ICO_V[a] + i * _ICO_V[b] + j * _ICO_V[c]
            pts.append(p / np.linalg.norm(p))
        return idx

    tris = []
    for f in range(20):
        for j in range(nf):
            for i in range(nf - j):
                tris.append((vid(f, i, j), vid(f, i + 1, j), vid(f, i, j + 1)))
                if i + j + 2 <= nf:
                    tris.append((vid(f, i + 1, j), vid(f, i + 1, j + 1), vid(f, i, j + 1)))
    verts = np.array(pts, dtype=np.float64)
    tris = np.array(tris, dtype=np.int32)
    return verts, tris


def sphere_subdivisions(radius_lambda: float, target_edge_lambda: float = 1.0 / 9.0) -> int:
    """Face subdivision nf whose mean edge is closest to the target edge."""
    guess = max(1, int(round(radius_lambda * 1.203 / target_edge_lambda)))
    best = None
    for nf in range(max(1, guess - 3), guess + 4):
        v, t = _geodesic_unit(nf)
        err = abs(_mean_edge(v * radius_lambda, t) - target_edge_lambda)
        if best is None or err < best[0]:
            best = (err, nf)
    return best[1]


def sphere_mesh(radius_lambda: float, freq_hz: float, nf: int | None = None,
                jitter_seed: int | None = None, name: str = "") -> Mesh:
    """Geodesic PEC sphere of radius ``radius_lambda`` wavelengths."""
    lam = wavelength(freq_hz)
    if nf is None:
        nf = sphere_subdivisions(radius_lambda)
    v, t = _geodesic_unit(nf)
    vl = v * radius_lambda
    if jitter_seed is not None:
        ebar = _mean_edge(vl, t)
        rng = np.random.default_rng(jitter_seed)
        vl = vl + (0.02 * ebar / math.sqrt(3.0)) * rng.uniform(-1.0, 1.0, size=vl.shape)
        vl = vl * (radius_lambda / np.linalg.norm(vl, axis=1))[:, None]
    return Mesh(verts=vl * lam, tris=t, freq_hz=float(freq_hz),
                name=name or f"sphere{radius_lambda:g}")
