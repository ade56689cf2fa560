"""The host planner (mesh validation, RWG table, grid, anchors, near-zone
pattern) built for the CPU with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, no GPU code) and run on valid and invalid meshes: no sanitizer report,
the plans equal the oracle's, and invalid meshes raise the documented
statuses. CPU only."""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import aim as oaim
from oracle.rwg import build_rwg
from workloads import plate_mesh, sphere_mesh

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1010_1456_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


def _record(f, verts, tris, freq, h=0.1, order=2, rn=0.3):
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    f.write(np.int64(v.shape[0]).tobytes())
    f.write(v.tobytes())
    f.write(np.int64(t.shape[0]).tobytes())
    f.write(t.tobytes())
    f.write(np.float64(freq).tobytes())
    f.write(np.float64(h).tobytes())
    f.write(np.int32(order).tobytes())
    f.write(np.float64(rn).tobytes())


def _digests(mesh, h=0.1, M=2, rn=0.3):
    rwg = build_rwg(mesh.verts, mesh.tris)
    g = oaim.grid_plan(rwg.verts, h * mesh.lam, M)
    anc = oaim.anchors(g, rwg.centre).ravel()
    ip, ix = oaim.near_pairs(rwg.centre, rn * mesh.lam)
    i = np.arange(anc.size)
    sa = int(np.sum((i % 7 + 1) * anc))
    j = np.arange(ix.size)
    sc = int(np.sum((j % 13 + 1) * ix))
    n = np.arange(rwg.n)
    se = int(np.sum((n % 5 + 1) * (rwg.edge[:, 0] + 3 * rwg.edge[:, 1] + 5 * rwg.tplus
                                   + 7 * rwg.tminus)))
    return rwg.n, ix.size, [int(v) for v in g.n], sa, sc, se


@pytest.fixture(scope="module")
def driver():
    gxx = shutil.which("g++")
    if not gxx or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "host_plan_sanitize")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-I", CSRC,
                    os.path.join(HERE, "host_plan_sanitize.cpp"), os.path.join(CSRC, "host_plan.cpp"),
                    "-o", exe, "-lpthread"], check=True, capture_output=True)
    yield exe, d
    shutil.rmtree(d, ignore_errors=True)


def test_host_planner_under_sanitizers(driver):
    exe, d = driver
    good = [plate_mesh(1.0, 0.3e9), plate_mesh(4.0, 1.2e9, jitter_seed=1002),
            sphere_mesh(1.0, 0.3e9, nf=11), sphere_mesh(2.0, 0.6e9, nf=22, jitter_seed=1005)]
    p = plate_mesh(1.0, 0.3e9)
    bad_index = p.tris.copy()
    bad_index[5, 1] = p.verts.shape[0]
    three = np.concatenate([p.tris, p.tris[:1]])  # an edge shared by three triangles
    flat = p.tris.copy()
    flat[3] = [flat[3, 0], flat[3, 0], flat[3, 1]]  # zero-area triangle
    bad = [(p.verts, bad_index, p.freq_hz, -2), (p.verts, three, p.freq_hz, -2),
           (p.verts, flat, p.freq_hz, -2), (p.verts, p.tris, -1.0, -1)]
    path = os.path.join(d, "meshes.bin")
    with open(path, "wb") as f:
        for m in good:
            _record(f, m.verts, m.tris, m.freq_hz)
        for v, t, fr, _ in bad:
            _record(f, v, t, fr)
        _record(f, p.verts, p.tris, p.freq_hz, order=7)  # order outside 1..5
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    out = r.stdout.split("\n")
    for m, line in zip(good, out):
        f = line.split()
        assert f[0] == "ok", line
        n, nnz, grid, sa, sc, se = _digests(m)
        assert int(f[1]) == n and int(f[2]) == nnz
        assert [int(v) for v in f[3:6]] == grid
        assert all(int(P) >= 2 * g - 1 for P, g in zip(f[6:9], grid))
        assert (int(f[9]), int(f[10]), int(f[11])) == (sa, sc, se)
    for (_, _, _, status), line in zip(bad, out[len(good):]):
        assert line == f"error {status}", line
    assert out[len(good) + len(bad)] == "error -1"
