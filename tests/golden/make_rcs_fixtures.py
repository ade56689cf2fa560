#!/usr/bin/env python3
"""Write the oracle's bistatic RCS of the benchmark scatterers (FP64, CPU).

Test infrastructure: this script calls only the FP64 oracle (``oracle/``)
and the seeded input generators (``workloads/``); nothing it stores comes
from the GPU library. Each case solves the AIM system of one scatterer with
the oracle's restarted GMRES (right Jacobi, Section 2.2) to a tolerance a
hundred times tighter than the GPU solves' 1e-4, then evaluates
sigma_theta_theta (the quantity of eq. (1)) on the 2-degree grid of
``oracle.farfield.rcs_grid(2.0)``: theta = 0, 2, ..., 180 degrees (91 rows) by
phi = 0, 2, ..., 358 degrees (180 columns). The GPU solve tests compare their
sigma_theta_theta with these through err_theta_theta, eq. (1).

Cases (workloads of the benchmark configurations; AIM with h = 0.1 lambda,
M = 2, near radius 0.3 lambda):

  plate16      16-lambda plate at 4.8 GHz, EFIE, x-polarised wave toward -z
               (Section 2.1); oracle tolerance 1e-6
  sphere8      8-lambda-radius sphere at 2.4 GHz, CFIE with alpha = 0.6 (the
               paper's formulation for closed bodies, Section 2.2), same wave;
               oracle tolerance 1e-6 (about an hour of CPU time, once)
  b6plate4     the jittered 4-lambda plate of the uneven batch (0.3 GHz, seed
               1002), EFIE, two oblique waves
  b6sphere2    the jittered 2-lambda-radius sphere of the uneven batch
               (0.3 GHz, seed 1005), CFIE alpha = 0.6, the same two waves

Oblique waves (arrival direction theta_i, phi_i = 0): theta_i = 2 pi/7 with
theta-hat polarisation and theta_i = 5 pi/7 with phi-hat polarisation, two of
the batch's sixteen.

Usage:  python tests/golden/make_rcs_fixtures.py CASE [CASE ...]
Writes tests/golden/rcs_<case>[_w<i>].txt.gz.
"""

from __future__ import annotations

import gzip
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OBLIQUE = [(2.0 * math.pi / 7.0, 0.0, 0), (5.0 * math.pi / 7.0, 0.0, 1)]
NORMAL = [(0.0, 0.0, 0)]

CASES = {
    # name: (mesh recipe, formulation alpha (None = EFIE), waves, oracle tol, GMRES cap)
    "plate16": (("config", "plate16"), None, NORMAL, 1e-6, 4000),
    "sphere8": (("config", "sphere8"), 0.6, NORMAL, 1e-6, 2000),
    "b6plate4": (("batch6", 1), None, OBLIQUE, 1e-6, 2000),
    "b6sphere2": (("batch6", 4), 0.6, OBLIQUE, 1e-6, 2000),
}


def fixture_path(case: str, wave: int) -> str:
    n = len(CASES[case][2])
    return os.path.join(HERE, f"rcs_{case}.txt.gz" if n == 1 else f"rcs_{case}_w{wave}.txt.gz")


def load_fixture(path: str):
    """(sigma (91, 180), metadata dict) of a fixture file."""
    meta = {}
    with gzip.open(path, "rt") as f:
        for line in f:
            if not line.startswith("#"):
                break
            if ":=" in line:
                k, v = line[1:].split(":=", 1)
                v = v.strip()
                if v.startswith("np.float64(") and v.endswith(")"):  # numpy scalar repr
                    v = v[len("np.float64("):-1]
                meta[k.strip()] = v
    sigma = np.loadtxt(path)
    return sigma, meta


def _mesh(recipe):
    from workloads import config_mesh, config_meshes

    kind, arg = recipe
    return config_mesh(arg) if kind == "config" else config_meshes("batch6")[arg]


_G = {}


def _sigma_rows(args):
    theta_rows, I = args
    from oracle import farfield as off

    return off.sigma_tt(_G["rwg"], _G["k"], I, theta_rows, _G["phi"])


def run_case(case: str, workers: int) -> None:
    import scipy.fft

    from oracle import aim as oaim
    from oracle import excitation as oexc
    from oracle import farfield as off
    from oracle import mfie as omfie
    from oracle.constants import wavenumber
    from oracle.gmres import gmres
    from oracle.rwg import build_rwg

    recipe, alpha, waves, tol, cap = CASES[case]
    t0 = time.time()
    mesh = _mesh(recipe)
    rwg = build_rwg(mesh.verts, mesh.tris)
    k = wavenumber(mesh.freq_hz)
    print(f"[{case}] N={rwg.n}: building the oracle operator", flush=True)
    op = oaim.build_operator(rwg, k, 0.1 * mesh.lam, 2, 0.3 * mesh.lam, cfie_alpha=alpha)
    print(f"[{case}] operator built in {time.time() - t0:.0f} s (nnz {op.near.nnz})", flush=True)
    pad = tuple(int(2 * v) for v in op.grid.n)
    theta, phi = off.rcs_grid(2.0)
    with scipy.fft.set_workers(workers):
        ghat = oaim.green_spectrum(k, op.grid, pad)
        for wi, (th_i, ph_i, pol) in enumerate(waves):
            if alpha is None:
                b = oexc.planewave_rhs(rwg, k, th_i, ph_i, pol)
            else:
                b = omfie.planewave_rhs_c(rwg, k, th_i, ph_i, pol, alpha)
            t1 = time.time()
            count = [0]

            def apply_a(v):
                count[0] += 1
                if count[0] % 20 == 0:
                    print(f"[{case}] wave {wi}: {count[0]} products, {time.time() - t1:.0f} s",
                          flush=True)
                return oaim.matvec_fft(op, v, pad=pad, ghat=ghat)

            x, info = gmres(apply_a, b, op.zmom_diag, tol, restart=100, max_iter=cap)
            print(f"[{case}] wave {wi}: {info['iters']} iterations, residual {info['resid']:.3e}, "
                  f"{time.time() - t1:.0f} s", flush=True)
            if not info["converged"]:
                raise SystemExit(f"{case}: the oracle solve did not reach {tol}")
            t2 = time.time()
            _G.update(rwg=rwg, k=k, phi=phi)
            chunks = np.array_split(theta, max(1, min(len(theta), 4 * workers)))
            with mp.get_context("fork").Pool(workers) as pool:
                parts = pool.map(_sigma_rows, [(c, x) for c in chunks])
            sigma = np.concatenate(parts, axis=0)
            print(f"[{case}] wave {wi}: sigma in {time.time() - t2:.0f} s", flush=True)
            form = "EFIE" if alpha is None else f"CFIE alpha={alpha}"
            header = "\n".join([
                f"Oracle bistatic sigma_theta_theta (m^2) of {mesh.name}, {form}, AIM h=0.1 lambda,",
                "M=2, near radius 0.3 lambda; the quantity whose relative RMS difference is",
                "err_theta_theta, eq. (1) (Section 2.2). Rows theta = 0..180 deg step 2,",
                "columns phi = 0..358 deg step 2. Written by tests/golden/make_rcs_fixtures.py,",
                "which calls only oracle/ and workloads/.",
                f"case := {case}",
                f"mesh := {mesh.name}",
                f"freq_hz := {mesh.freq_hz!r}",
                f"n := {rwg.n}",
                f"cfie_alpha := {alpha if alpha is not None else 'none'}",
                f"wave := {th_i!r} {ph_i!r} {pol}",
                f"oracle_tol := {tol!r}",
                f"oracle_iterations := {int(info['iters'])}",
                f"oracle_residual := {float(info['resid'])!r}",
            ])
            path = fixture_path(case, wi)
            with gzip.open(path, "wt") as f:
                np.savetxt(f, sigma, fmt="%.10e", header=header)
            print(f"[{case}] wrote {path}", flush=True)


def main(argv):
    cases = argv or list(CASES)
    workers = int(os.environ.get("FIXTURE_WORKERS", str(os.cpu_count() or 1)))
    for c in cases:
        if c not in CASES:
            raise SystemExit(f"unknown case {c}; choose from {sorted(CASES)}")
        run_case(c, workers)


if __name__ == "__main__":
    main(sys.argv[1:])
