"""The benchmark workloads, by name.

Each entry fixes the scatterer, frequency and AIM parameters of one workload:
grid spacing h (in wavelengths), stencil order M, near-zone radius (in
wavelengths) and the GMRES tolerance.

* ``plate1``: 1-lambda plate at 0.3 GHz, 9x9 squares, 225 unknowns.
* ``plate16``: 16-lambda plate at 4.8 GHz, 144x144 squares, 61,920 unknowns.
* ``sphere8``: 8-lambda sphere at 2.4 GHz, nf=87, 227,070 unknowns.
* ``batch6``: plates of side 2, 4, 8 lambda and spheres of radius 1, 2, 4
  lambda, each jittered (seeds 1001..1006), 16 plane waves each.
* ``plate128``: 128-lambda plate at 38.4 GHz, 1152x1152 squares.
"""

from __future__ import annotations

from .meshes import plate_mesh, sphere_mesh

_BASE = dict(h_lambda=0.1, order=2, near_radius_lambda=0.3)

CONFIGS = {
    "plate1": dict(_BASE, kind="plate", size=1.0, freq_hz=0.3e9, tol=1e-6),
    "plate16": dict(_BASE, kind="plate", size=16.0, freq_hz=4.8e9, tol=1e-4),
    "sphere8": dict(_BASE, kind="sphere", size=8.0, freq_hz=2.4e9, tol=1e-4),
    "plate128": dict(_BASE, kind="plate", size=128.0, freq_hz=38.4e9, tol=1e-4),
    "batch6": dict(_BASE, kind="batch", tol=1e-4, members=[
        ("plate", 2.0, 1001), ("plate", 4.0, 1002), ("plate", 8.0, 1003),
        ("sphere", 1.0, 1004), ("sphere", 2.0, 1005), ("sphere", 4.0, 1006)]),
}

# sphere face subdivisions for the configured radii (mean edge closest to
# lambda/9; ``workloads.meshes.sphere_subdivisions`` recomputes them)
SPHERE_NF = {1.0: 11, 2.0: 22, 4.0: 43, 8.0: 87}


def _member(kind, size, freq_hz, seed=None):
    if kind == "plate":
        return plate_mesh(size, freq_hz, jitter_seed=seed)
    return sphere_mesh(size, freq_hz, nf=SPHERE_NF.get(size), jitter_seed=seed)


def config_mesh(name: str):
    c = CONFIGS[name]
    if c["kind"] == "batch":
        raise ValueError("batch config: use config_meshes")
    return _member(c["kind"], c["size"], c["freq_hz"])


def config_meshes(name: str, freq_hz: float = 0.3e9):
    """Meshes of a (possibly batched) config. Batch members share one
    frequency; their sizes are in wavelengths."""
    c = CONFIGS[name]
    if c["kind"] != "batch":
        return [config_mesh(name)]
    return [_member(k, s, freq_hz, seed) for (k, s, seed) in c["members"]]
