#!/usr/bin/env python3
"""AIM matvec throughput and HBM roofline on one MI355X.

A step is one AIM product y = Z x of the hot path: precision staging of the
c128 solver vector, projection, pruned forward FFT passes, the x pass with the
Green's spectrum multiply, pruned inverse passes, interpolation fused with the
near-zone correction. The headline is the mixed path (c64 arithmetic on c128
vectors, as the solver applies it) on the 8-lambda PEC sphere; the FP64 path
is timed on the same input beside it. Per-kernel durations come from HIP events
recorded between the kernels of every timed product. The FP64 CPU oracle is
timed on a bounded sample on the host for reference.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere8]
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "AIM matvec/s + % HBM roofline, mixed vs FP64 at equal RCS err (sphere 8λ)"
STAGES = ["projection", "fwd_z", "fwd_y", "x_green", "inv_y", "inv_z", "interp_near"]
# kernel of each stage on the mixed path (the projection's depends on the tuned variant)
KERNELS = [None, "k_fft_contig<float, false", "k_fft_strided<float, false", "k_fft_mid<float",
           "k_fft_strided<float, true", "k_fft_contig<float, true", "k_interp_near<float"]


def stage_kernel(d, fused):
    if d == 0:
        return "k_anterp_fftz<float" if fused else "k_anterp_gather<float"
    return KERNELS[d]


CSRC = os.path.join(ROOT, "paper_1010_1456_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
CAL_BYTES = 256 << 20  # the --calibrate kernel reads and writes 256 MiB per launch


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# sources that define the product's kernels, their launches and the layout of
# the operator data they read (the solver, RCS, ABI glue, host planning and
# near-field quadrature do not change a product kernel's memory traffic)
MATVEC_SOURCES_EXCLUDED = ("api.hip", "solver.hip", "rcs.hip", "host_plan.cpp", "geom_device.h")


def sources_digest():
    """Digest of the product's kernel sources: HBM counters taken on other
    sources are stale."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip", ".cpp")) and name not in MATVEC_SOURCES_EXCLUDED:
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()


def short_kernel(name):
    name = name.replace("(anonymous namespace)::", "").split("(")[0]
    name = re.sub(r"^void |aim::|fftk::", "", name)
    name = re.sub(r"HIP_vector_type<(\w+), 2u>", r"\1", name)
    name = re.sub(r"vec2_of<(\w+)>::type", r"\1", name)
    return name.strip()


def ingest_pmc(fetch_csv, write_csv, workload):
    """Per-kernel HBM bytes per dispatch from a FETCH_SIZE run and a WRITE_SIZE
    run of `bench.py --calibrate`: each counter is scaled by what it reads for
    the calibration kernel (a plain elementwise multiply that reads 256 MiB
    and writes 256 MiB). Writes profiles/<workload>_kernel_traffic.json."""
    def load(path):
        acc = {}
        for r in csv.DictReader(open(path)):
            acc.setdefault(short_kernel(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}

    fetch, nf = load(fetch_csv)
    write, _ = load(write_csv)
    cal = [k for k in fetch if "MulFunctor" in k]
    if not cal:
        raise SystemExit("no calibration kernel in the counter runs (run bench.py with --calibrate)")
    fs = CAL_BYTES / (fetch[cal[0]] * 1024.0)
    ws = CAL_BYTES / (write[cal[0]] * 1024.0)
    kernels = {}
    for k, f in fetch.items():
        if not k.startswith("k_"):
            continue
        w = write.get(k, 0.0)
        kernels[k] = {"dispatches": nf[k], "fetch_kib": f, "write_kib": w,
                      "read_bytes": f * 1024.0 * fs, "write_bytes": w * 1024.0 * ws,
                      "bytes": (f * fs + w * ws) * 1024.0}
    out = {"workload": workload, "sources_sha256": sources_digest(),
           "fetch_scale": fs, "write_scale": ws,
           "calibration": f"{cal[0]}: reads and writes {CAL_BYTES} bytes per launch",
           "counters": [os.path.basename(fetch_csv), os.path.basename(write_csv)],
           "kernels": kernels}
    path = os.path.join(PROFILES, f"{workload}_kernel_traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(f"wrote {path}: FETCH_SIZE x {fs:.3f}, WRITE_SIZE x {ws:.3f}")
    for k, v in sorted(kernels.items()):
        print(f"  {k}: read {v['read_bytes'] / 1e6:.1f} MB, write {v['write_bytes'] / 1e6:.1f} MB")


def measured_traffic(workload, kernel_prefix):
    """HBM bytes per launch of the kernel from the committed counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(PROFILES, f"{workload}_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha256") != sources_digest():
        return None
    hits = [v for k, v in t["kernels"].items() if k.startswith(kernel_prefix)]
    return float(hits[0]["bytes"]) if len(hits) == 1 else None


def stage_bytes(info, mesh, nrhs, s_grid, s_real, s_x, s_y, path):
    """Algorithmic HBM bytes of each step of one product: every operator datum
    read once, vectors read/written once, grid fields per the pruned passes:
    the projection writes and the interpolation reads the occupied nodes only
    (O of them, on L z lines), the z passes move the L occupied lines, the
    forward y pass reads their rows and the inverse y pass writes them."""
    n = info["n"][mesh]
    nnz = info["nnz"][mesh]
    K = (info["order"] + 1) ** 3
    Nx, Ny, Nz = info["grid"][mesh]
    Px, Py, Pz = info["pad"][mesh]
    V2 = Nx * Py * Pz
    O, L = info["occ_nodes"][mesh], info["occ_lines"][mesh]
    F = 4 * nrhs
    H = (Px // 2 + 1) * (Py // 2 + 1) * (Pz // 2 + 1)
    lam = n * (4 * K * s_real + 4)
    curl = 3 * n * K * s_real if info["cfie_alpha"][mesh] is not None else 0.0  # combined field
    if info["planar_z"][mesh] >= 0:  # scatterer in one grid plane: everything on that plane
        A1, A2 = Nx * Ny, Nx * Py
        H2 = (Px // 2 + 1) * (Py // 2 + 1)
        lam2 = n * (4 * (info["order"] + 1) ** 2 * s_real + 4)
        return np.array([
            F * O * s_grid + lam2 + nrhs * n * s_x,
            0.0,
            F * (A1 + A2) * s_grid,
            2 * F * A2 * s_grid + H2 * s_grid,
            F * (A2 + A1) * s_grid,
            0.0,
            F * O * s_grid + lam2 + nnz * (s_grid + 4) + 4 * (n + 1) + nrhs * n * (s_x + s_y),
        ], dtype=np.float64)
    if info["fused_projection"][mesh][path]:  # projection inside the forward z pass
        proj, fwdz = lam + nrhs * n * s_x + F * L * Pz * s_grid, 0.0
    else:
        proj, fwdz = F * O * s_grid + lam + nrhs * n * s_x, F * L * (Nz + Pz) * s_grid
    return np.array([
        proj,                                                          # projection (+ forward z)
        fwdz,                                                          # forward z
        F * (L * Pz + V2) * s_grid,                                    # forward y
        2 * F * V2 * s_grid + H * s_grid,                              # x pass + spectrum
        F * (V2 + L * Pz) * s_grid,                                    # inverse y
        F * L * (Pz + Nz) * s_grid,                                    # inverse z
        F * O * s_grid + lam + nnz * (s_grid + 4) + 4 * (n + 1)
        + nrhs * n * (s_x + s_y) + curl,                               # interp + near
    ], dtype=np.float64)


def fill_report(info):
    """Set-up (matrix fill) phase times of the plan, summed over scatterers,
    and the near-zone fill rate: FP64 entries of Z^MOM - Z^grid per second."""
    ph = {k: float(sum(d[k] for d in info["setup_ms"])) for k in info["setup_ms"][0]}
    out = {f"{k}_ms": v for k, v in ph.items()}
    out["near_entries"] = int(info["nnz_total"])
    out["near_entries_per_s"] = info["nnz_total"] / (ph["near_fill"] * 1e-3) if ph["near_fill"] > 0 else None
    return out


def cpu_fill_baseline(cfg, freq_hz):
    """The oracle's near-zone fill (Z^MOM on the pattern, then Z^grid) on a
    half-wavelength-radius sphere meshed at the workload's density: FP64
    entries per second on one host core (numpy)."""
    from oracle import aim as oaim
    from oracle import mom as omom
    from oracle.constants import wavenumber
    from oracle.rwg import build_rwg
    from workloads import sphere_mesh

    m = sphere_mesh(0.5, freq_hz)
    rwg = build_rwg(m.verts, m.tris)
    k = wavenumber(freq_hz)
    grid = oaim.grid_plan(rwg.verts, cfg["h_lambda"] * m.lam, cfg["order"])
    anc = oaim.anchors(grid, rwg.centre)
    lam = oaim.projection(rwg, grid, anc)
    indptr, indices = oaim.near_pairs(rwg.centre, cfg["near_radius_lambda"] * m.lam)
    rows = np.repeat(np.arange(rwg.n), np.diff(indptr))
    t0 = time.perf_counter()
    omom.sparse_z(rwg, k, indptr, indices)
    oaim.zgrid_entries(k, grid, lam, anc, rows, indices)
    dt = time.perf_counter() - t0
    return {"near_entries_per_s": indices.shape[0] / dt, "seconds": dt, "cores": 1, "kind": "oracle",
            "sample": (f"near-zone fill of a 0.5-lambda-radius sphere (N={rwg.n}, {indices.shape[0]} "
                       f"entries, M={cfg['order']}) by oracle.mom.sparse_z and oracle.aim.zgrid_entries")}


def time_path(plan, A, prec, x, y, steps, warmup):
    import torch

    if warmup > 0:
        plan.matvec_timed(x, y, prec, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stage_ms, total_ms = plan.matvec_timed(x, y, prec, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, stage_ms / steps, total_ms


def cpu_baseline(mesh, cfg, nrhs, pad, cfie_alpha=None):
    """The FP64 oracle's FFT-form product on the host cores (one product)."""
    import scipy.fft
    import scipy.sparse

    from oracle import aim as oaim
    from oracle.constants import wavenumber
    from oracle.rwg import build_rwg
    from workloads import random_current

    cores = max(1, min(16, os.cpu_count() or 1))
    k = wavenumber(mesh.freq_hz)
    t_setup = time.perf_counter()
    rwg = build_rwg(mesh.verts, mesh.tris)
    grid = oaim.grid_plan(rwg.verts, cfg["h_lambda"] * mesh.lam, cfg["order"])
    anc = oaim.anchors(grid, rwg.centre)
    lam = oaim.projection(rwg, grid, anc)
    indptr, indices = oaim.near_pairs(rwg.centre, cfg["near_radius_lambda"] * mesh.lam)
    near = scipy.sparse.csr_matrix((np.ones(indices.shape[0], dtype=np.complex128), indices, indptr),
                                   shape=(rwg.n, rwg.n))
    op = oaim.AIMOperator(rwg=rwg, k=k, grid=grid, anc=anc, lam=lam, near=near,
                          zmom_diag=np.ones(rwg.n, dtype=np.complex128))
    if cfie_alpha is not None:
        op.curl = oaim.curl_projection(rwg, grid, anc)
        op.alpha = cfie_alpha
    with scipy.fft.set_workers(cores):
        ghat = oaim.green_spectrum(k, grid, pad)
        log(f"[cpu_baseline] oracle set-up {time.perf_counter() - t_setup:.1f} s")
        x = random_current(rwg.n, nrhs=nrhs, seed=7)
        t0 = time.perf_counter()
        oaim.matvec_fft(op, x, pad=pad, ghat=ghat)
        dt = time.perf_counter() - t0
    return {
        "value": 1.0 / dt, "unit": "matvec/s", "cores": cores, "kind": "oracle",
        "seconds_per_matvec": dt,
        "sample": (f"one FP64 FFT-form AIM product (oracle.aim.matvec_fft) on the full workload "
                   f"(N={rwg.n}, grid {tuple(int(v) for v in grid.n)} padded {tuple(pad)}), "
                   f"scipy.fft with {cores} workers; near-zone values set to 1 on the oracle's "
                   f"own near pattern ({indices.shape[0]} nnz; the sparse product's cost does not "
                   f"depend on the values)"),
    }


def solve_compare(plan, A, mesh, workload, iters):
    """The x-polarised wave toward -z solved by both paths (GMRES(100), Jacobi,
    tol 1e-4, fixed iteration budget): time per iteration, residuals, and the
    RCS agreement err_tt(mixed, fp64) on a 2-degree grid; for spheres also
    err_tt against the Mie series."""
    import torch

    from oracle import farfield as off
    from oracle import mie as omie
    from oracle.constants import wavenumber
    from workloads import planewave_set

    th, ph = off.rcs_grid(2.0)
    waves = ([tuple(w) for w in planewave_set(8)] if workload == "batch6" else [(0.0, 0.0, 0)])
    for prec in (A.AIM_MIXED, A.AIM_FP64):  # warm-up: work buffers, first launches
        plan.solve(waves, prec, tol=1e-4, restart=100, max_iter=2, raise_on_noconv=False)
    res = {}
    for name, prec in (("mixed", A.AIM_MIXED), ("fp64", A.AIM_FP64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = plan.solve(waves, prec, tol=1e-4, restart=100, max_iter=iters,
                           raise_on_noconv=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sig = plan.rcs(x, th, ph)[:, 0]  # first wave, every scatterer
        res[name] = dict(seconds=dt, iterations=st[0]["iterations"], residual=st[0]["residual"],
                         converged=st[0]["converged"], matvec_low=st[0]["matvec_low"],
                         matvec_fp64=st[0]["matvec_fp64"], ms_per_iteration=dt / max(1, st[0]["iterations"]) * 1e3,
                         sigma=sig)
        log(f"[bench] solve {name}: {st[0]['iterations']} its, residual {st[0]['residual']:.3e}, {dt:.2f} s")
    out = {k: {kk: vv for kk, vv in v.items() if kk != "sigma"} for k, v in res.items()}
    out["err_tt_mixed_vs_fp64"] = max(off.err_tt(a, b, th)
                                      for a, b in zip(res["mixed"]["sigma"], res["fp64"]["sigma"]))
    if workload.startswith("sphere"):
        k = wavenumber(mesh.freq_hz)
        sm = omie.sigma_tt(k, float(workload[len("sphere"):]) * mesh.lam, th, ph)
        for name in ("mixed", "fp64"):
            out[name]["err_tt_vs_mie"] = off.err_tt(res[name]["sigma"][0], sm, th)
    out["mixed_speedup_per_iteration"] = res["fp64"]["ms_per_iteration"] / res["mixed"]["ms_per_iteration"]
    out["setting"] = (f"GMRES(100), right Jacobi, tol 1e-4, at most {iters} iterations, "
                      + ("16 plane waves per scatterer (theta_i = i pi/7, both polarisations)"
                         if workload == "batch6" else "x-pol wave toward -z"))
    return out


def accuracy_sweep(A, max_iter):
    """err_tt of AIM solutions against references, the form of the paper's
    Tables 1-2 err columns (Section 2.2) with this library's parameters: a
    4-lambda plate (EFIE) and a 1-lambda-radius sphere at 0.3 GHz, x-polarised
    wave toward -z, 2-degree RCS grid. References: the classical MOM solution
    (every basis pair in the near zone, so the product is Z^MOM), the
    fifth-order AIM (the paper's reference where MOM is too costly) and, for
    the sphere, the Mie series. Candidates sweep the stencil order M, the
    near-zone size gamma (in grid spacings) and the grid spacing h."""
    import torch

    from oracle import farfield as off
    from oracle import mie as omie
    from oracle.constants import wavenumber
    from workloads import plate_mesh, sphere_mesh

    th, ph = off.rcs_grid(2.0)
    wave = [(0.0, 0.0, 0)]
    f = 0.3e9
    scatterers = [("plate4", plate_mesh(4.0, f), None), ("sphere1", sphere_mesh(1.0, f), 1.0)]
    out = {"setting": "GMRES(100), right Jacobi; candidates tol 1e-4, references tol 1e-8; "
                      "err_tt per eq. (1) over a 2-degree (theta, phi) grid", "scatterers": []}
    for name, m, radius in scatterers:
        ext = np.ptp(m.verts, axis=0)
        r_all = 1.01 * float(np.linalg.norm(ext)) / m.lam + 0.05  # every pair near

        def run(order, h, near_lambda, prec, tol):
            t0 = time.perf_counter()
            plan = A.Plan([(m.verts, m.tris, m.freq_hz)], h_lambda=h, order=order,
                          near_radius_lambda=near_lambda)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            plan.solve(wave, prec, tol=tol, restart=100, max_iter=2, raise_on_noconv=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = plan.solve(wave, prec, tol=tol, restart=100, max_iter=max_iter,
                               raise_on_noconv=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sig = plan.rcs(x, th, ph)[0, 0]
            info = plan.info()
            plan.close()
            return sig, dict(n=int(info["n_total"]), grid=[int(v) for v in info["grid"][0]],
                             nnz=int(info["nnz_total"]), setup_s=setup, iterations=st[0]["iterations"],
                             converged=bool(st[0]["converged"]), residual=float(st[0]["residual"]),
                             solve_s=dt)

        log(f"[sweep] {name}: references")
        refs, ref_meta = {}, {}
        refs["mom"], ref_meta["mom"] = run(2, 0.1, r_all, A.AIM_FP64, 1e-8)
        refs["aim_m5"], ref_meta["aim_m5"] = run(5, 0.1, 0.5, A.AIM_FP64, 1e-8)
        if radius is not None:
            refs["mie"] = omie.sigma_tt(wavenumber(f), radius * m.lam, th, ph)
        ref_meta["aim_m5"]["params"] = "M=5, h=0.1 lambda, gamma=5"
        ref_meta["aim_m5"]["err_vs"] = {k: off.err_tt(refs["aim_m5"], v, th)
                                        for k, v in refs.items() if k != "aim_m5"}
        ref_meta["mom"]["err_vs"] = {k: off.err_tt(refs["mom"], v, th)
                                     for k, v in refs.items() if k not in ("mom", "aim_m5")}
        cand = [(M, 0.1, 3.0, p) for M in (1, 2, 3, 4, 5) for p in ("mixed", "fp64")]
        cand += [(2, 0.1, g, "mixed") for g in (2.0, 4.0, 5.0)]
        cand += [(2, hh, 3.0, "mixed") for hh in (0.075, 0.125, 0.15)]
        cand += [(3, 0.1, 4.0, "mixed"), (4, 0.1, 5.0, "mixed")]
        rows = []
        for M, hh, g, p in cand:
            prec = A.AIM_MIXED if p == "mixed" else A.AIM_FP64
            sig, meta = run(M, hh, g * hh, prec, 1e-4)
            meta.update(M=M, h_lambda=hh, gamma=g, precision=p,
                        err_vs={k: off.err_tt(sig, v, th) for k, v in refs.items()})
            rows.append(meta)
            log(f"[sweep] {name} M={M} h={hh} gamma={g} {p}: its {meta['iterations']}, "
                + ", ".join(f"err vs {k} {v:.2e}" for k, v in meta["err_vs"].items()))
        out["scatterers"].append(dict(name=name, references=ref_meta, rows=rows))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sphere8",
                    choices=["sphere8", "plate16", "plate1", "plate128", "batch6"])
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides per scatterer (default 1; 16 for batch6)")
    ap.add_argument("--order", type=int, default=None,
                    help="stencil order M (default: the workload's, 2)")
    ap.add_argument("--cfie", type=float, default=None, metavar="ALPHA",
                    help="solve the combined-field equation alpha EFIE + (1 - alpha) eta MFIE "
                         "on the closed scatterers (the paper's alpha is 0.6; open ones keep "
                         "the EFIE) instead of the EFIE")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--solve-iters", type=int, default=300,
                    help="GMRES iteration budget of the solve comparison (0 skips it)")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain elementwise copy of 256 MiB (3 launches) whose "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the HBM byte counts")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the throughput line, print the accuracy/parameter sweep "
                         "(err_tt against MOM, fifth-order AIM and Mie references) as one JSON line")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter_collection.csv of a FETCH_SIZE and a WRITE_SIZE "
                         "rocprofv3 run of `bench.py --calibrate` into "
                         "profiles/<workload>_kernel_traffic.json, then exit")
    args = ap.parse_args(argv)
    if args.ingest_pmc:
        ingest_pmc(args.ingest_pmc[0], args.ingest_pmc[1], args.workload)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1010_1456_amd import aim as A
    from workloads import CONFIGS, config_mesh, config_meshes, random_current

    if args.sweep:
        print(json.dumps(accuracy_sweep(A, 3000)), flush=True)
        return
    if args.calibrate:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del a, b
    cfg = dict(CONFIGS[args.workload])
    if args.order is not None:
        cfg["order"] = args.order
    log(f"[bench] meshing {args.workload}")
    meshes = config_meshes(args.workload)
    mesh = meshes[0]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    plan = A.Plan([(m.verts, m.tris, m.freq_hz) for m in meshes], h_lambda=cfg["h_lambda"],
                  order=cfg["order"], near_radius_lambda=cfg["near_radius_lambda"],
                  cfie_alpha=args.cfie, cfie_closed_only=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = plan.info()
    n = info["n_total"]
    log(f"[bench] set-up {setup_s:.2f} s: N={n} grid={info['grid'][0]} pad={info['pad'][0]} "
        f"nnz={info['nnz_total']}")
    R = args.nrhs if args.nrhs is not None else (16 if args.workload == "batch6" else 1)
    x = torch.from_numpy(random_current(n, nrhs=R, seed=7)).cuda()
    y = torch.empty_like(x)

    res = {}
    for name, prec, sg, sr, path in (("mixed", A.AIM_MIXED_IO64, 8, 4, 1), ("fp64", A.AIM_FP64, 16, 8, 0)):
        log(f"[bench] timing {name}: {args.warmup} warm-up + {args.steps} products")
        wall, st_ms, tot_ms = time_path(plan, A, prec, x, y, args.steps, args.warmup)
        b = sum(stage_bytes(info, mi, R, sg, sr, 16, 16, path) for mi in range(info["nmesh"]))
        res[name] = dict(wall=wall, stage_ms=st_ms, total_ms=tot_ms, bytes=b)
        log(f"[bench] {name}: {wall / args.steps * 1e3:.3f} ms/product, stages(ms)="
            + ",".join(f"{v:.3f}" for v in st_ms))

    mx = res["mixed"]
    fused = bool(info["fused_projection"][0][1])  # (first scatterer's variant names the kernel)
    ms_per_step = mx["wall"] / args.steps * 1e3
    value = R * args.steps / mx["wall"]
    d = int(np.argmax(mx["stage_ms"]))
    achieved = mx["bytes"][d] / (mx["stage_ms"][d] * 1e-3) / 1e9
    total_bytes = float(mx["bytes"].sum())
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: " + {
                "sphere8": "PEC sphere radius 8 lambda at 2.4 GHz, geodesic mesh nf=87 (151,380 "
                           "triangles)",
                "plate16": "PEC plate 16 lambda at 4.8 GHz, 144x144 squares (41,472 triangles)",
                "plate1": "PEC plate 1 lambda at 0.3 GHz, 9x9 squares (162 triangles)",
                "plate128": "PEC plate 128 lambda at 38.4 GHz, 1152x1152 squares",
                "batch6": "6 scatterers in one plan at 0.3 GHz: PEC plates 2, 4, 8 lambda and spheres "
                          "1, 2, 4 lambda (seeded vertex jitter), R right-hand sides each",
            }[args.workload] + f"; {'EFIE' if args.cfie is None else f'CFIE (alpha {args.cfie})'}-AIM h={cfg['h_lambda']} lambda, M={cfg['order']} ({(cfg['order'] + 1) ** 3}-node "
                               f"stencils), near radius {cfg['near_radius_lambda']} lambda; "
                               f"N={n}, grid {info['grid'] if info['nmesh'] > 1 else info['grid'][0]}, "
                               f"FFT {info['pad'] if info['nmesh'] > 1 else info['pad'][0]}, "
                               f"near nnz {info['nnz_total']}; nrhs={R}"),
            "systems_per_product": info["nmesh"] * R,
            "precision": "c64 grid/stencil/near arithmetic on c128 vectors (mixed path)",
            "fused_projection": info["fused_projection"][0][1],
            "gather_nodes_per_wave": info["gather_npw"][0][1],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": stage_kernel(d, fused) + f"> ({STAGES[d]})",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.workload, stage_kernel(d, fused)),
            "algorithmic_bytes_per_launch": float(mx["bytes"][d]),
            "avg_launch_ms": float(mx["stage_ms"][d]),
        },
        "matvec_roofline": {
            "algorithmic_bytes": total_bytes,
            "achieved_GBs": total_bytes / (mx["wall"] / args.steps) / 1e9,
            "frac": total_bytes / (mx["wall"] / args.steps) / 1e9 / HBM_PEAK_GBS,
        },
        "stage_ms": {s: float(v) for s, v in zip(STAGES, mx["stage_ms"])},
        "stage_GBs": {s: float(b / (v * 1e-3) / 1e9) for s, b, v in zip(STAGES, mx["bytes"], mx["stage_ms"])
                      if b > 0},
        "fp64": {
            "value": R * args.steps / res["fp64"]["wall"],
            "ms_per_step": res["fp64"]["wall"] / args.steps * 1e3,
            "algorithmic_bytes": float(res["fp64"]["bytes"].sum()),
            "frac": float(res["fp64"]["bytes"].sum()) / (res["fp64"]["wall"] / args.steps) / 1e9
            / HBM_PEAK_GBS,
            "stage_ms": {s: float(v) for s, v in zip(STAGES, res["fp64"]["stage_ms"])},
        },
        "mixed_over_fp64": res["fp64"]["wall"] / mx["wall"],
        "setup_s": setup_s,
        "fill": fill_report(info),
        "device_bytes": info["device_bytes"],
    }
    if args.solve_iters > 0:
        out["solve"] = solve_compare(plan, A, mesh, args.workload, args.solve_iters)
        if args.workload.startswith("sphere") and args.cfie is None:
            # the paper's formulation for the closed sphere: CFIE, alpha = 0.6
            log("[bench] CFIE (alpha 0.6) plan for the solve comparison")
            plan_c = A.Plan([(m.verts, m.tris, m.freq_hz) for m in meshes], h_lambda=cfg["h_lambda"],
                            order=cfg["order"], near_radius_lambda=cfg["near_radius_lambda"],
                            cfie_alpha=0.6)
            out["solve_cfie"] = solve_compare(plan_c, A, mesh, args.workload, args.solve_iters)
            out["solve_cfie"]["setting"] = "CFIE alpha 0.6; " + out["solve_cfie"]["setting"]
            plan_c.close()
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(mesh, cfg, R, tuple(info["pad"][0]), args.cfie)
        out["fill"]["cpu_oracle"] = cpu_fill_baseline(cfg, mesh.freq_hz)
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
