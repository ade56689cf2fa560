"""aim_rcs_noalloc, the RCS for callers that cannot allocate: through the C
ABI, on a plan whose allocator refuses every request once set-up is done, two
calls in a row (the second with fewer directions and right-hand sides) equal
aim_rcs (FP64, relative 1e-12 of the largest sigma), allocate nothing, and
sizes beyond the fixed scratch are refused."""

import ctypes
import math
import sys

import numpy as np
import pytest

from workloads import plate_mesh, random_current, sphere_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


class GateAllocator:
    """torch caching-allocator memory until `deny` is set, NULL after."""

    def __init__(self):
        from paper_1010_1456_amd import aim as A

        self.deny = False
        self.calls_denied = 0

        def _alloc(ctx, nbytes, stream):
            if self.deny:
                self.calls_denied += 1
                return None
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0)))

        def _free(ctx, ptr, stream):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._a = A.ALLOC_FN(_alloc)
        self._f = A.FREE_FN(_free)
        self.struct = A.AimAllocator(None, self._a, self._f)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _grid(step_deg):
    th = np.deg2rad(np.arange(0.0, 180.0 + 1e-9, step_deg))
    ph = np.deg2rad(np.arange(0.0, 360.0 - 1e-9, step_deg))
    return th, ph


def test_rcs_noalloc_matches_rcs_without_allocating():
    from paper_1010_1456_amd import aim as A

    torch.cuda.set_device(0)
    meshes = [sphere_mesh(2.0, 0.3e9, nf=22), plate_mesh(1.0, 0.3e9, jitter_seed=9)]
    L = A.lib()
    keep = []
    arr = (A.AimMesh * 2)()
    for i, m in enumerate(meshes):
        arr[i] = A._mesh_struct(m.verts, m.tris, m.freq_hz, keep)
    p = A._params(0.1, 2, 0.3)
    gate = GateAllocator()
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream()
    _log("[no_alloc] set-up")
    assert L.aim_setup(arr, 2, ctypes.byref(p), ctypes.byref(gate.struct),
                       ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)) == A.AIM_OK
    inf = A.AimInfo()
    assert L.aim_plan_info(h, ctypes.byref(inf)) == A.AIM_OK
    n = inf.n_total
    try:
        calls = [(2, 1.0), (1, 5.0)]  # (right-hand sides, grid step in degrees)
        x = torch.from_numpy(random_current(n, nrhs=2, seed=17)).cuda()
        refs, outs, dirs = [], [], []
        for nrhs, step in calls:
            th, ph = _grid(step)
            ref = np.zeros((2, nrhs, th.size, ph.size))
            assert L.aim_rcs(h, nrhs, ctypes.c_void_p(x.data_ptr()), th.size,
                             th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ph.size,
                             ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ctypes.c_void_p(stream.cuda_stream)) == A.AIM_OK
            refs.append(ref)
            dirs.append((torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()))
            outs.append(torch.full((2, nrhs, th.size, ph.size), math.nan, dtype=torch.float64,
                                   device="cuda"))
        # 2 x 1 x 65,160 directions: more partial sums than the scratch holds
        # for the sphere's 17 point chunks, so that call runs with fewer chunks
        assert 2 * 181 * 360 * math.ceil(7 * 20 * 22 * 22 / 4096) > A.AIM_RCS_SCRATCH_ELEMS
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        gate.deny = True
        for (nrhs, step), (tht, pht), out in zip(calls, dirs, outs):
            _log(f"[no_alloc] call nrhs={nrhs} step={step}")
            st = L.aim_rcs_noalloc(h, nrhs, ctypes.c_void_p(x.data_ptr()), tht.numel(),
                                   ctypes.c_void_p(tht.data_ptr()), pht.numel(),
                                   ctypes.c_void_p(pht.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(stream.cuda_stream))
            assert st == A.AIM_OK, L.aim_last_error()
        torch.cuda.synchronize()
        assert gate.calls_denied == 0
        assert torch.cuda.memory_allocated() == before
        for ref, out in zip(refs, outs):
            got = out.cpu().numpy()
            assert np.isfinite(got).all()
            for mi in range(2):
                err = np.abs(got[mi] - ref[mi]).max() / np.abs(ref[mi]).max()
                assert err <= 1e-12, (mi, err)
        # beyond the scratch: refused, nothing launched
        big = torch.zeros(1025, dtype=torch.float64, device="cuda")
        st = L.aim_rcs_noalloc(h, 1, ctypes.c_void_p(x.data_ptr()), 1025, ctypes.c_void_p(big.data_ptr()),
                               1025, ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(outs[0].data_ptr()),
                               ctypes.c_void_p(stream.cuda_stream))
        assert st == A.AIM_ERR_ARG and b"scratch" in L.aim_last_error()
        assert gate.calls_denied == 0
    finally:
        gate.deny = False
        torch.cuda.synchronize()
        L.aim_destroy(h)


def test_rcs_noalloc_binding_rejects_bad_arguments():
    from paper_1010_1456_amd import aim as A

    m = plate_mesh(1.0, 0.3e9)
    plan = A.Plan([(m.verts, m.tris, m.freq_hz)])
    x = torch.zeros((1, plan.n_total), dtype=torch.complex128, device="cuda")
    th = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        plan.rcs_noalloc(x, th.float(), th)
    with pytest.raises(ValueError):
        plan.rcs_noalloc(x, th, th, out=torch.zeros((1, 1, 3, 2), dtype=torch.float64, device="cuda"))
    s = plan.rcs_noalloc(x, th, th)
    torch.cuda.synchronize()
    assert tuple(s.shape) == (1, 1, 3, 3) and float(s.abs().max()) == 0.0
    plan.close()
