#!/usr/bin/env python3
"""AIM matvec throughput and HBM roofline on one MI355X.

A step is one AIM product y = Z x of the hot path: precision staging of the
c128 solver vector, projection, pruned forward FFT passes, the x pass with the
Green's spectrum multiply, pruned inverse passes, interpolation fused with the
near-zone correction. The headline is the mixed path (c64 arithmetic on c128
vectors, as the solver applies it) on the 8-lambda PEC sphere with the paper's
formulation for closed bodies, the combined-field equation with alpha = 0.6
(the EFIE operator is timed beside it as a reference line); the FP64 path
is timed on the same input beside it. The rate comes from HIP events around a
HIP graph of K products (median of several launches); per-kernel durations from
HIP events recorded between the kernels of a second pass of K products. The
FP64 CPU oracle's product is timed on the host cores for reference.

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


def measured_traffic(workload, kernel_prefix, row=None):
    """HBM bytes per launch of the kernel from the committed counter summary, or
    None when there is none or the kernel sources changed since it was taken.
    row: the tile-row variant (bytes) of the x and strided passes in use (the
    counter runs also see the set-up tuner's other variant)."""
    path = os.path.join(PROFILES, f"{workload}_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha256") != sources_digest():
        return None
    hits = [k for k in t["kernels"] if k.startswith(kernel_prefix)]
    if len(hits) > 1 and row is not None:
        hits = [k for k in hits if re.search(rf", {int(row)}(, (true|false))?>$", k)]
    return float(t["kernels"][hits[0]]["bytes"]) if len(hits) == 1 else None


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


def x_pass_flops(info, nrhs):
    """Algorithmic floating-point operations of the x pass of one product,
    summed over the scatterers: per line a forward and an inverse complex FFT
    of the padded length P (5 P log2 P each, the radix-2 count) and the
    spectrum multiply (6 P); lines = fields x P_y x P_z (P_y only for a
    scatterer in one grid plane)."""
    total = 0.0
    for mesh in range(info["nmesh"]):
        Px, Py, Pz = info["pad"][mesh]
        lines = 4 * nrhs * Py * (1 if info["planar_z"][mesh] >= 0 else Pz)
        total += lines * (2 * 5 * Px * np.log2(Px) + 6 * Px)
    return total


# FP32 vector peak of the chip's units without packed-FP32 instructions (the
# build disables them): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz;
# the vendor's 157.3 TFLOP/s counts packed FP32
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FP32_VECTOR_TFLOPS = 157.3


def pipelined_bytes(info, mesh, path, b):
    """With the y, x and y passes pipelined in one kernel (aim_info.xy_groups
    > 1) their stage boundaries fall together and the forward y step carries
    the time of all three: so does its byte count."""
    if info["xy_groups"][mesh][path] > 1:
        b = b.copy()
        b[2] += b[3] + b[4]
        b[3] = b[4] = 0.0
    return b


def x_pass_alu(info, nrhs, ms):
    """The x pass is bound by vector-ALU issue rather than HBM: its FLOP rate
    against the FP32 vector peaks."""
    fl = x_pass_flops(info, nrhs)
    tf = fl / (ms * 1e-3) / 1e12
    return {"bound": "alu", "flops_per_launch": fl, "avg_launch_ms": float(ms),
            "achieved_TFLOPs": tf,
            "peak_TFLOPs_nonpacked": FP32_NONPACKED_TFLOPS, "frac_nonpacked": tf / FP32_NONPACKED_TFLOPS,
            "peak_TFLOPs_vector": FP32_VECTOR_TFLOPS, "frac_vector": tf / FP32_VECTOR_TFLOPS,
            "convention": "2 x 5 P log2 P + 6 P per line (forward and inverse FFT, spectrum multiply)"}


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


def time_path(plan, A, prec, x, y, steps, warmup, launches):
    """The product timed as a HIP graph of `steps` products, launched
    `launches` times with events around each launch (median reported), and a
    second pass of `steps` direct products with events between the kernels
    for the per-step times. Returns (graph ms per launch, stage ms per
    product, wall seconds around the graph launches)."""
    import torch

    for _ in range(warmup):
        plan.matvec(x, prec, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launch_ms = plan.matvec_graph_timed(x, y, prec, steps, launches)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, _ = plan.matvec_timed(x, y, prec, steps)
    torch.cuda.synchronize()
    return launch_ms, stage_ms / steps, wall


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """HBM bandwidth of a plain device-to-device copy of nbytes (read + write
    counted), median of reps timed copies after one warm-up: the measured
    ceiling the product's kernels are also compared with."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        out.append(2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    return float(np.median(out))


def host_cpu():
    """(cores this process may run on, CPU model name)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        cores = min(cores, int(omp))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, cores), model


def cpu_baseline(mesh, cfg, nrhs, pad, cfie_alpha=None):
    """The FP64 oracle's FFT-form product (oracle.aim.matvec_fft) on the host:
    on every core available to the process (median of 5 after one warm-up),
    and on one thread (one product after the warm-up)."""
    import scipy.fft
    import scipy.sparse

    from oracle import aim as oaim
    from oracle.constants import wavenumber
    from oracle.rwg import build_rwg
    from workloads import random_current

    cores, model = host_cpu()
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
    x = random_current(rwg.n, nrhs=nrhs, seed=7)
    with scipy.fft.set_workers(cores):
        ghat = oaim.green_spectrum(k, grid, pad)
        log(f"[cpu_baseline] oracle set-up {time.perf_counter() - t_setup:.1f} s, {cores} cores")
        oaim.matvec_fft(op, x, pad=pad, ghat=ghat)  # warm-up
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            oaim.matvec_fft(op, x, pad=pad, ghat=ghat)
            times.append(time.perf_counter() - t0)
    with scipy.fft.set_workers(1):
        t0 = time.perf_counter()
        oaim.matvec_fft(op, x, pad=pad, ghat=ghat)
        t1 = time.perf_counter() - t0
    dt = float(np.median(times))
    return {
        "value": nrhs / dt, "unit": "matvec/s", "cores": cores, "kind": "oracle",
        "cpu_model": model, "os_cpu_count": os.cpu_count(),
        "seconds_per_matvec": dt, "seconds_per_matvec_runs": times,
        "one_thread": {"value": nrhs / t1, "seconds_per_matvec": t1},
        "sample": (f"the whole workload, not sampled: FP64 FFT-form AIM product "
                   f"(oracle.aim.matvec_fft) with N={rwg.n}, grid {tuple(int(v) for v in grid.n)} "
                   f"padded {tuple(pad)}, {nrhs} right-hand side(s); scipy.fft and BLAS on {cores} "
                   f"threads, median of 5 after one warm-up; the one-thread figure is one product "
                   f"after the warm-up. Near-zone values are 1 on the oracle's own near pattern "
                   f"({indices.shape[0]} nnz): the sparse product's cost does not depend on them, "
                   f"and the oracle's fill of the true values takes about an hour"),
    }


def oracle_fixture(workload):
    """(sigma_tt, metadata) the oracle wrote for this workload's
    normal-incidence solve (tests/golden), or None."""
    import gzip

    path = os.path.join(ROOT, "tests", "golden", f"rcs_{workload}.txt.gz")
    if not os.path.exists(path):
        return None
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
    return np.loadtxt(path), meta


def solve_compare(plan, A, mesh, workload, iters, alpha):
    """The workload's plane waves solved by both paths (GMRES(100), Jacobi,
    tol 1e-4 on the FP64 residual, at most `iters` iterations): time, systems
    solved per second, iterations, residuals, and the RCS agreement
    err_tt(mixed, fp64) on a 2-degree grid; against the oracle's solve where
    a stored oracle RCS exists, and for spheres against the Mie series."""
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
    nsys = plan.nmesh * len(waves)
    for name, prec in (("mixed", A.AIM_MIXED), ("fp64", A.AIM_FP64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = plan.solve(waves, prec, tol=1e-4, restart=100, max_iter=iters,
                           raise_on_noconv=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sig = plan.rcs(x, th, ph)  # (mesh, wave, theta, phi)
        its = [q["iterations"] for q in st]
        conv = all(q["converged"] for q in st)
        res[name] = dict(seconds=dt, systems=nsys, systems_per_s=nsys / dt,
                         iterations=max(its), converged=conv,
                         residual=max(q["residual"] for q in st),
                         matvec_low=st[0]["matvec_low"], matvec_fp64=st[0]["matvec_fp64"],
                         ms_per_iteration=dt / max(1, max(its)) * 1e3, sigma=sig)
        if nsys > 1:
            res[name]["per_mesh"] = [
                dict(mesh=mi, max_iterations=max(q["iterations"] for q in st if q["mesh"] == mi),
                     max_residual=max(q["residual"] for q in st if q["mesh"] == mi),
                     converged=all(q["converged"] for q in st if q["mesh"] == mi))
                for mi in range(plan.nmesh)]
        log(f"[bench] solve {name}: {max(its)} its, worst residual {res[name]['residual']:.3e}, "
            f"{'converged' if conv else 'NOT converged'}, {dt:.2f} s")
    out = {k: {kk: vv for kk, vv in v.items() if kk != "sigma"} for k, v in res.items()}
    out["err_tt_mixed_vs_fp64"] = max(
        off.err_tt(a, b, th) for a, b in zip(res["mixed"]["sigma"].reshape(-1, *th.shape, *ph.shape),
                                             res["fp64"]["sigma"].reshape(-1, *th.shape, *ph.shape)))
    fx = oracle_fixture(workload) if nsys == 1 else None
    if fx is not None:
        for name in ("mixed", "fp64"):
            out[name]["err_tt_vs_oracle"] = off.err_tt(res[name]["sigma"][0, 0], fx[0], th)
        out["oracle"] = {k: fx[1][k] for k in ("oracle_tol", "oracle_iterations",
                                                "oracle_residual", "cfie_alpha")}
    if workload.startswith("sphere"):
        k = wavenumber(mesh.freq_hz)
        sm = omie.sigma_tt(k, float(workload[len("sphere"):]) * mesh.lam, th, ph)
        for name in ("mixed", "fp64"):
            out[name]["err_tt_vs_mie"] = off.err_tt(res[name]["sigma"][0, 0], sm, th)
    out["mixed_speedup"] = res["fp64"]["seconds"] / res["mixed"]["seconds"]
    out["setting"] = (("EFIE" if alpha is None else f"CFIE alpha {alpha} on closed scatterers, EFIE on "
                       "open ones") + f"; GMRES(100), right Jacobi, tol 1e-4, at most {iters} iterations, "
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


WORKLOAD_TEXT = {
    "sphere8": "PEC sphere radius 8 lambda at 2.4 GHz, geodesic mesh nf=87 (151,380 triangles)",
    "plate16": "PEC plate 16 lambda at 4.8 GHz, 144x144 squares (41,472 triangles)",
    "plate1": "PEC plate 1 lambda at 0.3 GHz, 9x9 squares (162 triangles)",
    "plate128": "PEC plate 128 lambda at 38.4 GHz, 1152x1152 squares",
    "batch6": "6 scatterers in one plan at 0.3 GHz: PEC plates 2, 4, 8 lambda and spheres 1, 2, 4 "
              "lambda (seeded vertex jitter), R right-hand sides each",
}


def measure_plan(plan, A, info, R, x, y, steps, warmup, launches):
    """Graph-timed throughput, per-step times and byte models of both paths."""
    res = {}
    for name, prec, sg, sr, path in (("mixed", A.AIM_MIXED_IO64, 8, 4, 1),
                                     ("fp64", A.AIM_FP64, 16, 8, 0)):
        log(f"[bench] timing {name}: {warmup} warm-up, {launches} graph launches of {steps} products")
        launch_ms, st_ms, wall = time_path(plan, A, prec, x, y, steps, warmup, launches)
        b = sum(pipelined_bytes(info, mi, path, stage_bytes(info, mi, R, sg, sr, 16, 16, path))
                for mi in range(info["nmesh"]))
        med = float(np.median(launch_ms))
        res[name] = dict(launch_ms=launch_ms, ms_per_step=med / steps, stage_ms=st_ms, bytes=b,
                         wall=wall, value=R * steps / (med * 1e-3))
        log(f"[bench] {name}: {med / steps:.4f} ms/product (graph, median of {launches}; launches "
            + ",".join(f"{v / steps:.4f}" for v in launch_ms) + "), stages(ms)="
            + ",".join(f"{v:.3f}" for v in st_ms))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--launches", type=int, default=5,
                    help="graph launches of --steps products each; the median is reported")
    ap.add_argument("--workload", default="sphere8",
                    choices=["sphere8", "plate16", "plate1", "plate128", "batch6"])
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides per scatterer (default 1; 16 for batch6)")
    ap.add_argument("--order", type=int, default=None,
                    help="stencil order M (default: the workload's, 2)")
    ap.add_argument("--cfie", type=float, default=0.6, metavar="ALPHA",
                    help="combination parameter of the combined-field equation alpha EFIE + "
                         "(1 - alpha) eta MFIE on the closed scatterers (the paper's is 0.6); "
                         "open ones keep the EFIE")
    ap.add_argument("--efie", action="store_true",
                    help="the EFIE on every scatterer (closed ones too)")
    ap.add_argument("--xy-groups", type=int, default=0, choices=[0, 1, 2, 4],
                    help="field groups of the pipelined y / x / y passes (0: chosen at set-up)")
    ap.add_argument("--member", type=int, default=None,
                    help="with a batch workload: time one of its scatterers alone "
                         "(same right-hand sides per scatterer)")
    ap.add_argument("--tile-rows", type=int, default=0, choices=[0, 64, 128],
                    help="bytes of grid lines per x / y pass tile (0: chosen at set-up)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-efie-line", action="store_true",
                    help="skip the EFIE reference line of a CFIE sphere workload")
    ap.add_argument("--solve-iters", type=int, default=3000,
                    help="GMRES iteration cap of the solve comparison (0 skips it)")
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
    from workloads import CONFIGS, config_meshes, random_current

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
    alpha = None if args.efie else args.cfie
    cfg = dict(CONFIGS[args.workload])
    if args.order is not None:
        cfg["order"] = args.order
    log(f"[bench] meshing {args.workload}")
    meshes = config_meshes(args.workload)
    if args.member is not None:  # one scatterer of a batch on its own
        if not 0 <= args.member < len(meshes):
            raise SystemExit(f"--member: {args.workload} has {len(meshes)} scatterers")
        meshes = [meshes[args.member]]
    mesh = meshes[0]
    torch.cuda.set_device(0)
    copy_gbs = copy_bandwidth()
    log(f"[bench] device-to-device copy: {copy_gbs:.0f} GB/s")

    R = args.nrhs if args.nrhs is not None else (16 if args.workload == "batch6" else 1)

    def make_plan(a):
        t0 = time.perf_counter()
        # the set-up times its kernel variants with the R right-hand sides per
        # mesh that the products below apply the operator to
        pl = A.Plan([(m.verts, m.tris, m.freq_hz) for m in meshes], h_lambda=cfg["h_lambda"],
                    order=cfg["order"], near_radius_lambda=cfg["near_radius_lambda"],
                    cfie_alpha=a, cfie_closed_only=True, xy_groups=args.xy_groups,
                    tile_rows=args.tile_rows, tune_rhs=min(R, 64) if R > 1 else 0)
        torch.cuda.synchronize()
        return pl, time.perf_counter() - t0

    plan, setup_s = make_plan(alpha)
    info = plan.info()
    n = info["n_total"]
    log(f"[bench] set-up {setup_s:.2f} s: N={n} grid={info['grid'][0]} pad={info['pad'][0]} "
        f"nnz={info['nnz_total']} cfie={info['cfie_alpha']} xy_groups={info['xy_groups']} "
        f"tile_bytes={info['tile_bytes']}")
    x = torch.from_numpy(random_current(n, nrhs=R, seed=7)).cuda()
    y = torch.empty_like(x)
    res = measure_plan(plan, A, info, R, x, y, args.steps, args.warmup, args.launches)

    mx = res["mixed"]
    fused = bool(info["fused_projection"][0][1])  # (first scatterer's variant names the kernel)
    piped = info["xy_groups"][0][1] > 1
    d = int(np.argmax(mx["stage_ms"]))
    kname = ("k_fft_xy<float> (fwd_y + x_green + inv_y pipelined over "
             f"{info['xy_groups'][0][1]} field groups)" if piped and d == 2
             else stage_kernel(d, fused) + f"> ({STAGES[d]})")
    achieved = mx["bytes"][d] / (mx["stage_ms"][d] * 1e-3) / 1e9
    total_bytes = float(mx["bytes"].sum())
    forms = sorted({"EFIE" if a is None else f"CFIE alpha={a}" for a in info["cfie_alpha"]})
    out = {
        "metric": METRIC,
        "value": mx["value"],
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}"
                         + (f" member {args.member} ({mesh.name}) alone" if args.member is not None else "")
                         + ": " + WORKLOAD_TEXT[args.workload]
                         + f"; {' and '.join(forms)}-AIM h={cfg['h_lambda']} lambda, M={cfg['order']} "
                         f"({(cfg['order'] + 1) ** 3}-node stencils), near radius "
                         f"{cfg['near_radius_lambda']} lambda; N={n}, grid "
                         f"{info['grid'] if info['nmesh'] > 1 else info['grid'][0]}, FFT "
                         f"{info['pad'] if info['nmesh'] > 1 else info['pad'][0]}, near nnz "
                         f"{info['nnz_total']}; nrhs={R}"),
            "systems_per_product": info["nmesh"] * R,
            "precision": "c64 grid/stencil/near arithmetic on c128 vectors (mixed path)",
            "timing": (f"HIP events around a HIP graph of {args.steps} products, median of "
                       f"{args.launches} launches after {args.warmup} direct products and one "
                       f"untimed launch; per-step times from a separate pass with events "
                       f"between the kernels"),
            "fused_projection": info["fused_projection"][0][1],
            "gather_nodes_per_wave": info["gather_npw"][0][1],
            "xy_pipeline_groups": info["xy_groups"][0][1],
            "tile_bytes_x_y": info["tile_bytes"][0][1],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.workload, "k_fft_xy<float" if piped and d == 2
                                        else stage_kernel(d, fused),
                                        row=(info["tile_bytes"][0][1][0] if d == 3 else
                                             info["tile_bytes"][0][1][1] if d in (2, 4) else None)),
            "algorithmic_bytes_per_launch": float(mx["bytes"][d]),
            "avg_launch_ms": float(mx["stage_ms"][d]),
            "copy_GBs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "x_pass_alu": x_pass_alu(info, R, mx["stage_ms"][3]) if mx["stage_ms"][3] > 0.01 else None,
        "matvec_roofline": {
            "algorithmic_bytes": total_bytes,
            "achieved_GBs": total_bytes / (mx["ms_per_step"] * 1e-3) / 1e9,
            "frac": total_bytes / (mx["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "frac_of_copy": total_bytes / (mx["ms_per_step"] * 1e-3) / 1e9 / copy_gbs,
        },
        "graph_launch_ms": [float(v) for v in mx["launch_ms"]],
        "stage_ms": {s_: float(v) for s_, v in zip(STAGES, mx["stage_ms"])},
        "stage_GBs": {s_: float(b / (v * 1e-3) / 1e9) for s_, b, v in zip(STAGES, mx["bytes"], mx["stage_ms"])
                      if b > 0 and v > 0},
        "fp64": {
            "value": res["fp64"]["value"],
            "ms_per_step": res["fp64"]["ms_per_step"],
            "graph_launch_ms": [float(v) for v in res["fp64"]["launch_ms"]],
            "algorithmic_bytes": float(res["fp64"]["bytes"].sum()),
            "frac": float(res["fp64"]["bytes"].sum()) / (res["fp64"]["ms_per_step"] * 1e-3) / 1e9
            / HBM_PEAK_GBS,
            "stage_ms": {s_: float(v) for s_, v in zip(STAGES, res["fp64"]["stage_ms"])},
        },
        "mixed_over_fp64": res["fp64"]["ms_per_step"] / mx["ms_per_step"],
        "setup_s": setup_s,
        "fill": fill_report(info),
        "device_bytes": info["device_bytes"],
    }
    if args.solve_iters > 0:
        out["solve"] = solve_compare(plan, A, mesh, args.workload, args.solve_iters, alpha)
    plan.close()
    if args.workload.startswith("sphere") and alpha is not None and not args.no_efie_line:
        # the EFIE operator on the same sphere, for reference: product rate and
        # the iterations its (mixed) solve needs to reach 1e-4, or the stall
        log("[bench] EFIE plan (reference line)")
        plan_e, _ = make_plan(None)
        info_e = plan_e.info()
        re_ = measure_plan(plan_e, A, info_e, R, x, y, args.steps, args.warmup, args.launches)
        out["efie"] = {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                           "frac": float(v["bytes"].sum()) / (v["ms_per_step"] * 1e-3) / 1e9
                           / HBM_PEAK_GBS} for k, v in re_.items()}
        if args.solve_iters > 0:
            import torch as _t

            plan_e.solve([(0.0, 0.0, 0)], A.AIM_MIXED, tol=1e-4, max_iter=2, raise_on_noconv=False)
            _t.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = plan_e.solve([(0.0, 0.0, 0)], A.AIM_MIXED, tol=1e-4, restart=100,
                                 max_iter=args.solve_iters, raise_on_noconv=False)
            _t.cuda.synchronize()
            out["efie"]["solve_mixed"] = dict(iterations=st[0]["iterations"],
                                              converged=st[0]["converged"],
                                              residual=st[0]["residual"],
                                              seconds=time.perf_counter() - t0,
                                              cap=args.solve_iters)
            log(f"[bench] EFIE solve: {st[0]['iterations']} its, residual {st[0]['residual']:.3e}")
        plan_e.close()
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(mesh, cfg, R, tuple(info["pad"][0]),
                                           info["cfie_alpha"][0])
        out["fill"]["cpu_oracle"] = cpu_fill_baseline(cfg, mesh.freq_hz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
