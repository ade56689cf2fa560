"""C ABI checks that need no GPU: exported symbols, host planning against the
oracle (bit-exact integer decisions), error paths."""

import os
import re

import numpy as np
import pytest

from oracle import aim as oaim
from oracle.rwg import build_rwg
from paper_1010_1456_amd import aim as lib_aim
from workloads import plate_mesh, sphere_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "aim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aim_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lib_aim.lib()
    declared = _declared_symbols()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(lib_aim.EXPORTED) == declared


def _compare_host_plan(mesh, h=0.1, M=2, rn=0.3):
    hp = lib_aim.host_plan(mesh.verts, mesh.tris, mesh.freq_hz, h, M, rn)
    rwg = build_rwg(mesh.verts, mesh.tris)
    g = oaim.grid_plan(rwg.verts, h * mesh.lam, M)
    anc = oaim.anchors(g, rwg.centre)
    ip, ix = oaim.near_pairs(rwg.centre, rn * mesh.lam)
    assert hp["n"] == rwg.n
    assert np.array_equal(hp["rwg"][:, 0:2], rwg.edge)
    assert np.array_equal(hp["rwg"][:, 2], rwg.tplus)
    assert np.array_equal(hp["rwg"][:, 3], rwg.tminus)
    assert np.array_equal(hp["rwg"][:, 4], rwg.vplus)
    assert np.array_equal(hp["rwg"][:, 5], rwg.vminus)
    assert np.array_equal(hp["grid"], g.n)
    assert np.array_equal(hp["x0"], g.x0)
    assert hp["h"] == g.h
    assert np.array_equal(hp["anchors"], anc)
    assert np.array_equal(hp["rowptr"], ip)
    assert np.array_equal(hp["cols"], ix)
    assert np.all(hp["pad"] >= 2 * hp["grid"] - 1)
    return hp


@pytest.mark.parametrize("mesh", [
    plate_mesh(1.0, 0.3e9), plate_mesh(4.0, 1.2e9, jitter_seed=1002), sphere_mesh(1.0, 0.3e9, nf=11),
    sphere_mesh(2.0, 0.6e9, nf=22, jitter_seed=1005)], ids=["plate1", "plate4j", "sphere1", "sphere2j"])
def test_host_plan_matches_oracle(mesh):
    _compare_host_plan(mesh)


def test_host_plan_plate16_counts():
    """16-lambda plate: 61,920 unknowns, 161x161x3 grid, near pattern equal
    to the oracle's (integer-exact)."""
    hp = _compare_host_plan(plate_mesh(16.0, 4.8e9))
    assert hp["n"] == 61920
    assert tuple(hp["grid"]) == (161, 161, 3)


def test_host_plan_other_orders():
    m = sphere_mesh(0.5, 0.3e9, nf=4)
    for M in (1, 3, 4, 5):
        _compare_host_plan(m, h=0.08, M=M, rn=0.25)


def test_error_paths():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=float)
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(v, np.array([[0, 1, 2], [0, 1, 3], [1, 0, 4]]), 0.3e9)
    assert e.value.status == lib_aim.AIM_ERR_MESH
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(v, np.array([[0, 1, 7]]), 0.3e9)
    assert e.value.status == lib_aim.AIM_ERR_MESH
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], float), np.array([[0, 1, 2]]), 0.3e9)
    assert e.value.status == lib_aim.AIM_ERR_MESH
    m = plate_mesh(1.0, 0.3e9)
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(m.verts, m.tris, -1.0)
    assert e.value.status == lib_aim.AIM_ERR_ARG
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(m.verts, m.tris, m.freq_hz, h_lambda=0.0)
    assert e.value.status == lib_aim.AIM_ERR_ARG
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(m.verts, m.tris, m.freq_hz, order=0)
    assert e.value.status == lib_aim.AIM_ERR_ARG
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(m.verts, m.tris, m.freq_hz, order=6)
    assert e.value.status == lib_aim.AIM_ERR_ARG
    # a single triangle has no interior edge
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(v[:3], np.array([[0, 1, 2]]), 0.3e9)
    assert e.value.status == lib_aim.AIM_ERR_MESH


def test_quadrature_points_parameter():
    """aim_params.quad_points: the paper's 7-point rule (7, or 0 for the
    same); any other count is refused before any work."""
    import ctypes

    L = lib_aim.lib()
    m = plate_mesh(1.0, 0.3e9)
    keep = []
    ms = lib_aim._mesh_struct(m.verts, m.tris, m.freq_hz, keep)
    for q, want in ((7, lib_aim.AIM_OK), (0, lib_aim.AIM_OK), (3, lib_aim.AIM_ERR_ARG),
                    (6, lib_aim.AIM_ERR_ARG), (-7, lib_aim.AIM_ERR_ARG)):
        p = lib_aim._params(0.1, 2, 0.3)
        p.quad_points = q
        hp = ctypes.c_void_p()
        st = L.aim_host_plan_build(ctypes.byref(ms), ctypes.byref(p), ctypes.byref(hp))
        assert st == want, (q, st)
        if st == lib_aim.AIM_OK:
            L.aim_host_plan_destroy(hp)
        else:
            assert "quad_points" in L.aim_last_error().decode()


def test_binding_layouts_and_constants_match_header(tmp_path):
    """The ctypes structures have the sizes and field offsets of the C
    declarations, and every #define the binding mirrors has the same value."""
    import ctypes
    import shutil
    import subprocess

    cc = shutil.which("g++") or shutil.which("gcc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"aim_info": lib_aim.AimInfo, "aim_params": lib_aim.AimParams,
               "aim_solve_opts": lib_aim.AimSolveOpts, "aim_solve_stats": lib_aim.AimSolveStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aim.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-x", "c", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, fname, val = ln.split()
        got[(cname, fname)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
    text = open(os.path.join(ROOT, "include", "aim.h")).read()
    defines = dict(re.findall(r"#define\s+(AIM_[A-Z0-9_]+)\s+(-?\d+)\b", text))
    for name, val in defines.items():
        if hasattr(lib_aim, name):
            assert getattr(lib_aim, name) == int(val), name
    enums = dict(re.findall(r"\b(AIM_[A-Z0-9_]+)\s*=\s*(-?\d+)", text))
    for name, val in enums.items():
        if hasattr(lib_aim, name):
            assert getattr(lib_aim, name) == int(val), name
    assert lib_aim.SETUP_PHASES[lib_aim.AIM_NSETUP - 1] == "tune"


def test_cfie_needs_a_closed_outward_mesh():
    """The combined field is accepted on a closed, outward-oriented sphere and
    refused on an open plate, on an inside-out sphere, on a sphere with one
    triangle flipped, and for alpha outside [0, 1]; the EFIE takes them all."""
    m = sphere_mesh(0.5, 0.3e9, nf=3)
    hp = lib_aim.host_plan(m.verts, m.tris, m.freq_hz, cfie_alpha=0.6)
    assert hp["n"] == 3 * m.tris.shape[0] // 2
    flipped_all = m.tris[:, ::-1].copy()
    flipped_one = m.tris.copy()
    flipped_one[5] = flipped_one[5, ::-1]
    p = plate_mesh(1.0, 0.3e9)
    bad = [(p.verts, p.tris, 0.6, lib_aim.AIM_ERR_MESH),
           (m.verts, flipped_all, 0.6, lib_aim.AIM_ERR_MESH),
           (m.verts, flipped_one, 0.6, lib_aim.AIM_ERR_MESH),
           (m.verts, m.tris, 1.5, lib_aim.AIM_ERR_ARG),
           (m.verts, m.tris, -0.1, lib_aim.AIM_ERR_ARG)]
    for verts, tris, alpha, status in bad:
        with pytest.raises(lib_aim.AimError) as e:
            lib_aim.host_plan(verts, tris, m.freq_hz, cfie_alpha=alpha)
        assert e.value.status == status
        lib_aim.host_plan(verts, tris, m.freq_hz)


def test_grid_size_limits():
    """Two triangles spanning 170 lambda need a 1703-node grid, whose padded
    length 3456 is the largest compiled FFT; 180 lambda needs more and is
    refused with AIM_ERR_ARG before anything is allocated."""
    tris = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)

    def square(side):
        return np.array([[0, 0, 0], [side, 0, 0], [side, side, 0], [0, side, 0]], dtype=float)

    hp = lib_aim.host_plan(square(170.0), tris, 0.3e9)
    assert list(hp["grid"]) == [1703, 1703, 3] and list(hp["pad"]) == [3456, 3456, 5]
    with pytest.raises(lib_aim.AimError) as e:
        lib_aim.host_plan(square(180.0), tris, 0.3e9)
    assert e.value.status == lib_aim.AIM_ERR_ARG
    assert "largest supported FFT length" in str(e.value)


def test_binding_rejects_bad_product_vectors():
    """The binding checks x and y before their pointers reach the library
    (which writes nrhs * n_total elements of y): dtype, contiguity, shape,
    size, overlap and device."""
    torch = pytest.importorskip("torch")
    n, dt = 10, torch.complex128
    x = torch.zeros((2, n), dtype=dt)
    cases = [
        (x.to(torch.complex64), None, "must be torch.complex128"),
        (torch.zeros((n, 2), dtype=dt).t(), None, "contiguous"),
        (torch.zeros((2, n + 1), dtype=dt), None, "shape"),
        (torch.zeros((2, 2, n), dtype=dt), None, "shape"),
        (torch.zeros((0, n), dtype=dt), None, "shape"),
        (x, torch.zeros((3, n), dtype=dt), "elements"),
        (x, torch.zeros((2, n), dtype=torch.complex64), "must be torch.complex128"),
        (x, x, "overlap"),
        (x[0], x[0:1].reshape(n), "overlap"),
        (x, torch.zeros((2, n), dtype=dt), "must be on cuda:0"),
        (x, None, "must be on cuda:0"),
    ]
    for xx, yy, msg in cases:
        with pytest.raises(ValueError, match=msg):
            lib_aim.check_vectors(xx, yy, n, dt, 0)
