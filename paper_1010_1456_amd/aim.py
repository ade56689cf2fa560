"""Python binding of libaim.so (ctypes; argument marshalling only).

Every step of the AIM product, the solve and the RCS runs in the library's
HIP kernels; PyTorch only supplies device memory (its caching allocator, via
the library's allocator callbacks) and streams. The names follow the C ABI in
include/aim.h.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaim.so")

AIM_OK = 0
AIM_ERR_ARG = -1
AIM_ERR_MESH = -2
AIM_ERR_HIP = -3
AIM_ERR_NOMEM = -4
AIM_ERR_NOCONV = -5
AIM_ERR_STATE = -6
AIM_FP64 = 0
AIM_MIXED = 1
AIM_MIXED_IO64 = 2
AIM_NSTAGE = 7
AIM_FLAG_NO_MIXED = 1
AIM_FLAG_CFIE = 2
AIM_FLAG_CFIE_CLOSED = 4
AIM_SOLVE_NO_GRAPH = 1
AIM_MAX_MESH = 16
AIM_DATA_LAMBDA64 = 1
AIM_DATA_NEAR64 = 2
AIM_DATA_ZDIAG64 = 3
AIM_DATA_GHAT64 = 4
AIM_DATA_CURL64 = 5
AIM_NSETUP = 5
AIM_RCS_SCRATCH_ELEMS = 1 << 20  # partial sums held by aim_rcs_noalloc's fixed array
# set-up phases of aim_info.setup_ms, in order
SETUP_PHASES = ("host_plan", "projection", "green", "near_fill", "tune")

EXPORTED = [
    "aim_setup", "aim_plan_info", "aim_destroy", "aim_matvec", "aim_matvec_timed",
    "aim_matvec_graph_timed", "aim_gmres_solve",
    "aim_excitation", "aim_rcs", "aim_rcs_noalloc", "aim_host_plan_build", "aim_host_plan_export",
    "aim_host_plan_destroy", "aim_export", "aim_debug_far_stage", "aim_debug_product_stage",
    "aim_last_error",
]


class AimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"aim status {status}: {msg}")
        self.status = status


class AimMesh(ctypes.Structure):
    _fields_ = [("nv", c_int64), ("verts", POINTER(c_double)), ("nt", c_int64),
                ("tris", POINTER(c_int32)), ("freq_hz", c_double)]


class AimParams(ctypes.Structure):
    _fields_ = [("h_lambda", c_double), ("order", c_int32), ("fft_min_pad", c_int32),
                ("near_radius_lambda", c_double), ("flags", c_int32), ("tuning", c_int32),
                ("cfie_alpha", c_double), ("quad_points", c_int32), ("reserved", c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)


class AimAllocator(ctypes.Structure):
    _fields_ = [("ctx", c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class AimPlanewave(ctypes.Structure):
    _fields_ = [("theta", c_double), ("phi", c_double), ("pol", c_int32), ("reserved", c_int32)]


class AimInfo(ctypes.Structure):
    M = AIM_MAX_MESH
    _fields_ = [("nmesh", c_int32), ("order", c_int32), ("n_total", c_int64),
                ("nnz_total", c_int64), ("n", c_int64 * M), ("offset", c_int64 * M),
                ("nnz", c_int64 * M), ("grid", (c_int32 * 3) * M), ("pad", (c_int32 * 3) * M),
                ("h", c_double * M), ("x0", (c_double * 3) * M), ("k", c_double * M),
                ("bytes_fp64", c_double * M), ("bytes_mixed", c_double * M),
                ("fused_projection", (c_int32 * 2) * M), ("planar_z", c_int32 * M),
                ("device_bytes", c_double), ("setup_ms", (c_double * AIM_NSETUP) * M),
                ("cfie_alpha", c_double * M), ("occ_nodes", c_int64 * M), ("occ_lines", c_int64 * M),
                ("gather_npw", (c_int32 * 2) * M), ("xy_groups", (c_int32 * 2) * M),
                ("tile_bytes", ((c_int32 * 2) * 2) * M)]


class AimSolveOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("restart", c_int32), ("max_iter", c_int32),
                ("warm_start", c_int32), ("flags", c_int32)]


class AimSolveStats(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("converged", c_int32), ("matvec_low", c_int32),
                ("matvec_fp64", c_int32), ("residual", c_double), ("seconds", c_double)]


_lib = None


def lib():
    """The loaded library. Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1010_1456_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "aim_setup": [POINTER(AimMesh), c_int32, POINTER(AimParams), POINTER(AimAllocator), P, POINTER(P)],
        "aim_plan_info": [P, POINTER(AimInfo)],
        "aim_matvec": [P, c_int32, c_int32, P, P, P],
        "aim_matvec_timed": [P, c_int32, c_int32, P, P, c_int32, POINTER(c_double),
                             POINTER(c_double), P],
        "aim_matvec_graph_timed": [P, c_int32, c_int32, P, P, c_int32, c_int32, POINTER(c_double),
                                   P],
        "aim_gmres_solve": [P, c_int32, c_int32, POINTER(AimPlanewave), POINTER(AimSolveOpts), P,
                            POINTER(AimSolveStats), P],
        "aim_excitation": [P, c_int32, POINTER(AimPlanewave), P, P],
        "aim_rcs": [P, c_int32, P, c_int32, POINTER(c_double), c_int32, POINTER(c_double),
                    POINTER(c_double), P],
        "aim_rcs_noalloc": [P, c_int32, P, c_int32, P, c_int32, P, P, P],
        "aim_host_plan_build": [POINTER(AimMesh), POINTER(AimParams), POINTER(P)],
        "aim_host_plan_export": [P, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32),
                                 POINTER(c_int32), POINTER(c_int64), POINTER(c_int32),
                                 POINTER(c_int32), POINTER(c_int32), POINTER(c_double)],
        "aim_export": [P, c_int32, c_int32, P, c_size_t],
        "aim_debug_far_stage": [P, c_int32, c_int32, c_int32, P, c_int32, P, P],
        "aim_debug_product_stage": [P, c_int32, c_int32, c_int32, P, c_int32, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = c_int32
    L.aim_destroy.argtypes = [P]
    L.aim_destroy.restype = None
    L.aim_host_plan_destroy.argtypes = [P]
    L.aim_host_plan_destroy.restype = None
    L.aim_last_error.argtypes = []
    L.aim_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check_vectors(x, y, n_total: int, dtype, device: int) -> int:
    """Validates the vectors of a product before their pointers reach the
    library, which writes nrhs * n_total elements of y: x (and y, if not
    None) must be contiguous tensors of `dtype` on GPU `device`, of shape
    (n_total,) or (nrhs, n_total), y of x's size. Returns nrhs."""
    for name, t in (("x", x), ("y", y)):
        if t is None:
            continue
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.dim() not in (1, 2) or t.shape[-1] != n_total or t.numel() == 0:
            raise ValueError(f"{name} must have shape (n_total,) or (nrhs, n_total) with "
                             f"n_total = {n_total}, got {tuple(t.shape)}")
    if y is not None:
        if y.numel() != x.numel():
            raise ValueError(f"y holds {y.numel()} elements, x {x.numel()}")
        xb, yb = x.data_ptr(), y.data_ptr()
        nb = x.numel() * x.element_size()
        if xb < yb + nb and yb < xb + nb:
            raise ValueError("x and y must not overlap")
    for name, t in (("x", x), ("y", y)):
        if t is not None and (not t.is_cuda or t.device.index != device):
            raise ValueError(f"{name} must be on cuda:{device}, got {t.device}")
    return x.numel() // n_total


def _check(status: int):
    if status != AIM_OK:
        raise AimError(status, lib().aim_last_error().decode())


def _mesh_struct(verts, tris, freq_hz, keep):
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    keep.extend([v, t])
    return AimMesh(v.shape[0], v.ctypes.data_as(POINTER(c_double)), t.shape[0],
                   t.ctypes.data_as(POINTER(c_int32)), float(freq_hz))


def _params(h_lambda, order, near_radius_lambda, fft_min_pad=0, flags=0, cfie_alpha=None,
            cfie_closed_only=False, xy_groups=0, tile_rows=0, tune_rhs=0):
    """tile_rows: 0 (chosen at set-up), 128 or 64 bytes of grid lines per
    tile of the x and strided y passes. tune_rhs: right-hand sides per mesh
    the set-up times the kernel variants with (0: one)."""
    if cfie_alpha is not None:
        flags |= AIM_FLAG_CFIE_CLOSED if cfie_closed_only else AIM_FLAG_CFIE
    rows = {0: 0, 128: 1, 64: 2}[int(tile_rows)]
    return AimParams(float(h_lambda), int(order), int(fft_min_pad), float(near_radius_lambda),
                     int(flags), int(xy_groups) | (rows << 8) | (int(tune_rhs) << 16),
                     float(cfie_alpha) if cfie_alpha is not None else 0.0, 7, 0)


def _waves(waves):
    arr = (AimPlanewave * len(waves))()
    for i, w in enumerate(waves):
        arr[i] = AimPlanewave(float(w[0]), float(w[1]), int(w[2]), 0)
    return arr


def host_plan(verts, tris, freq_hz, h_lambda=0.1, order=2, near_radius_lambda=0.3, fft_min_pad=0,
              cfie_alpha=None, cfie_closed_only=False):
    """Host phase only (no GPU): RWG table, anchors, near-zone CSR, grid."""
    L = lib()
    keep = []
    m = _mesh_struct(verts, tris, freq_hz, keep)
    p = _params(h_lambda, order, near_radius_lambda, fft_min_pad, cfie_alpha=cfie_alpha,
                cfie_closed_only=cfie_closed_only)
    hp = c_void_p()
    _check(L.aim_host_plan_build(ctypes.byref(m), ctypes.byref(p), ctypes.byref(hp)))
    try:
        n = c_int64()
        nnz = c_int64()
        _check(L.aim_host_plan_export(hp, ctypes.byref(n), ctypes.byref(nnz), None, None, None, None,
                                      None, None, None))
        rwg = np.zeros((n.value, 6), dtype=np.int32)
        anc = np.zeros((n.value, 3), dtype=np.int32)
        rowptr = np.zeros(n.value + 1, dtype=np.int64)
        cols = np.zeros(max(nnz.value, 1), dtype=np.int32)
        grid = np.zeros(3, dtype=np.int32)
        pad = np.zeros(3, dtype=np.int32)
        x0h = np.zeros(4, dtype=np.float64)
        _check(L.aim_host_plan_export(
            hp, None, None, rwg.ctypes.data_as(POINTER(c_int32)), anc.ctypes.data_as(POINTER(c_int32)),
            rowptr.ctypes.data_as(POINTER(c_int64)), cols.ctypes.data_as(POINTER(c_int32)),
            grid.ctypes.data_as(POINTER(c_int32)), pad.ctypes.data_as(POINTER(c_int32)),
            x0h.ctypes.data_as(POINTER(c_double))))
    finally:
        L.aim_host_plan_destroy(hp)
    return dict(n=n.value, nnz=nnz.value, rwg=rwg, anchors=anc, rowptr=rowptr,
                cols=cols[:nnz.value], grid=grid, pad=pad, x0=x0h[:3], h=x0h[3])


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator."""

    def __init__(self, device):
        import torch

        self._torch = torch
        self.device = device

        def _alloc(ctx, nbytes, stream):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                              int(stream or 0)))
            except Exception:  # out of memory -> NULL, reported by the library
                return None

        def _free(ctx, ptr, stream):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = AimAllocator(None, self._alloc, self._free)


class Plan:
    """An AIM operator on the current GPU for one or more meshes.

    meshes: list of (verts (nv,3) metres, tris (nt,3), freq_hz).
    tune_rhs: right-hand sides per mesh the set-up times the kernel variants
    with (the number the products will apply the operator to; 0: one)."""

    def __init__(self, meshes, h_lambda=0.1, order=2, near_radius_lambda=0.3, fft_min_pad=0,
                 mixed=True, stream=None, cfie_alpha=None, cfie_closed_only=False, xy_groups=0,
                 flags=0, tile_rows=0, tune_rhs=0):
        import torch

        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("the AIM library needs a GPU")
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        L = lib()
        keep = []
        arr = (AimMesh * len(meshes))()
        for i, (v, t, f) in enumerate(meshes):
            arr[i] = _mesh_struct(v, t, f, keep)
        p = _params(h_lambda, order, near_radius_lambda, fft_min_pad,
                    int(flags) | (0 if mixed else AIM_FLAG_NO_MIXED), cfie_alpha, cfie_closed_only,
                    xy_groups, tile_rows, tune_rhs)
        self._alloc = TorchAllocator(self.device)
        h = c_void_p()
        _check(L.aim_setup(arr, len(meshes), ctypes.byref(p), ctypes.byref(self._alloc.struct),
                           c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.nmesh = len(meshes)
        self._info = self.info()
        self.n_total = self._info["n_total"]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._torch.cuda.synchronize()
            lib().aim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = AimInfo()
        _check(lib().aim_plan_info(self._h, ctypes.byref(inf)))
        nm = inf.nmesh
        return dict(
            nmesh=nm, order=inf.order, n_total=inf.n_total, nnz_total=inf.nnz_total,
            n=[inf.n[i] for i in range(nm)], offset=[inf.offset[i] for i in range(nm)],
            nnz=[inf.nnz[i] for i in range(nm)], grid=[tuple(inf.grid[i]) for i in range(nm)],
            pad=[tuple(inf.pad[i]) for i in range(nm)], h=[inf.h[i] for i in range(nm)],
            x0=[tuple(inf.x0[i]) for i in range(nm)], k=[inf.k[i] for i in range(nm)],
            bytes_fp64=[inf.bytes_fp64[i] for i in range(nm)],
            bytes_mixed=[inf.bytes_mixed[i] for i in range(nm)],
            fused_projection=[(bool(inf.fused_projection[i][0]), bool(inf.fused_projection[i][1]))
                              for i in range(nm)],
            planar_z=[inf.planar_z[i] for i in range(nm)],
            device_bytes=inf.device_bytes,
            setup_ms=[dict(zip(SETUP_PHASES, inf.setup_ms[i])) for i in range(nm)],
            cfie_alpha=[None if inf.cfie_alpha[i] < 0 else inf.cfie_alpha[i] for i in range(nm)],
            occ_nodes=[inf.occ_nodes[i] for i in range(nm)],
            occ_lines=[inf.occ_lines[i] for i in range(nm)],
            gather_npw=[tuple(inf.gather_npw[i]) for i in range(nm)],
            xy_groups=[tuple(inf.xy_groups[i]) for i in range(nm)],
            tile_bytes=[tuple(tuple(inf.tile_bytes[i][q]) for q in range(2)) for i in range(nm)])

    def _stream(self, stream):
        s = stream if stream is not None else self._torch.cuda.current_stream()
        return c_void_p(s.cuda_stream)

    def matvec(self, x, precision=AIM_FP64, out=None, stream=None):
        """y = Z x for x of shape (n_total,) or (nrhs, n_total): complex128 for
        AIM_FP64 and AIM_MIXED_IO64, complex64 for AIM_MIXED (device tensors
        on the plan's GPU). `out`, if given, receives y and must match x."""
        torch = self._torch
        dt = torch.complex64 if precision == AIM_MIXED else torch.complex128
        nrhs = check_vectors(x, out, self.n_total, dt, self.device)
        xx = x.reshape(nrhs, self.n_total)
        y = out.reshape(nrhs, self.n_total) if out is not None else torch.empty_like(xx)
        _check(lib().aim_matvec(self._h, precision, nrhs, c_void_p(xx.data_ptr()),
                                c_void_p(y.data_ptr()), self._stream(stream)))
        return y.reshape(x.shape)

    def matvec_timed(self, x, y, precision, nrep, stream=None):
        """nrep products with HIP events between the kernels; returns
        (per-stage summed ms (AIM_NSTAGE,), first-to-last event ms)."""
        torch = self._torch
        dt = torch.complex64 if precision == AIM_MIXED else torch.complex128
        if y is None:
            raise ValueError("y is required")
        nrhs = check_vectors(x, y, self.n_total, dt, self.device)
        st = (c_double * AIM_NSTAGE)()
        tot = c_double()
        _check(lib().aim_matvec_timed(self._h, precision, nrhs, c_void_p(x.data_ptr()),
                                      c_void_p(y.data_ptr()), int(nrep), st, ctypes.byref(tot),
                                      self._stream(stream)))
        return np.array(st[:]), tot.value

    def matvec_graph_timed(self, x, y, precision, nrep, nlaunch=5, stream=None):
        """nrep products captured in one HIP graph, launched nlaunch times with
        events around each launch: returns the per-launch ms (nlaunch,)."""
        torch = self._torch
        dt = torch.complex64 if precision == AIM_MIXED else torch.complex128
        if y is None:
            raise ValueError("y is required")
        nrhs = check_vectors(x, y, self.n_total, dt, self.device)
        ms = (c_double * int(nlaunch))()
        _check(lib().aim_matvec_graph_timed(self._h, precision, nrhs, c_void_p(x.data_ptr()),
                                            c_void_p(y.data_ptr()), int(nrep), int(nlaunch), ms,
                                            self._stream(stream)))
        return np.array(ms[:])

    def excitation(self, waves, stream=None):
        torch = self._torch
        arr = _waves(waves)
        b = torch.empty((len(waves), self.n_total), dtype=torch.complex128, device="cuda")
        _check(lib().aim_excitation(self._h, len(waves), arr, c_void_p(b.data_ptr()),
                                    self._stream(stream)))
        return b

    def solve(self, waves, precision=AIM_MIXED, tol=1e-4, restart=100, max_iter=5000, x0=None,
              stream=None, raise_on_noconv=True, graphs=True):
        torch = self._torch
        arr = _waves(waves)
        R = len(waves)
        if x0 is not None:
            x = x0.to(torch.complex128).reshape(R, self.n_total).contiguous().clone()
        else:
            x = torch.zeros((R, self.n_total), dtype=torch.complex128, device="cuda")
        opts = AimSolveOpts(float(tol), int(restart), int(max_iter), 1 if x0 is not None else 0,
                            0 if graphs else AIM_SOLVE_NO_GRAPH)
        st = (AimSolveStats * (self.nmesh * R))()
        status = lib().aim_gmres_solve(self._h, precision, R, arr, ctypes.byref(opts),
                                       c_void_p(x.data_ptr()), st, self._stream(stream))
        if status != AIM_OK and (status != AIM_ERR_NOCONV or raise_on_noconv):
            _check(status)
        stats = [dict(mesh=i // R, wave=i % R, iterations=s.iterations, converged=bool(s.converged),
                      matvec_low=s.matvec_low, matvec_fp64=s.matvec_fp64, residual=s.residual,
                      seconds=s.seconds) for i, s in enumerate(st)]
        return x, stats

    def rcs(self, x, theta, phi, stream=None):
        """sigma_tt (nmesh, nrhs, ntheta, nphi) in m^2 for currents x (nrhs, n_total)."""
        torch = self._torch
        xx = x.reshape(-1, self.n_total).to(torch.complex128).contiguous()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        ph = np.ascontiguousarray(phi, dtype=np.float64)
        out = np.zeros((self.nmesh, xx.shape[0], th.size, ph.size), dtype=np.float64)
        _check(lib().aim_rcs(self._h, xx.shape[0], c_void_p(xx.data_ptr()), th.size,
                             th.ctypes.data_as(POINTER(c_double)), ph.size,
                             ph.ctypes.data_as(POINTER(c_double)),
                             out.ctypes.data_as(POINTER(c_double)), self._stream(stream)))
        return out

    def rcs_noalloc(self, x, theta, phi, out=None, stream=None):
        """aim_rcs_noalloc: sigma_tt (nmesh, nrhs, ntheta, nphi) on the device
        for currents x (nrhs, n_total) complex128 and directions theta, phi
        (float64 device tensors); asynchronous. `out` (float64 device tensor
        of that shape) receives it if given."""
        torch = self._torch
        nrhs = check_vectors(x, None, self.n_total, torch.complex128, self.device)
        for name, t in (("theta", theta), ("phi", phi)):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
                raise ValueError(f"{name} must be a contiguous 1-D float64 device tensor")
        shape = (self.nmesh, nrhs, theta.numel(), phi.numel())
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=x.device)
        elif (out.dtype != torch.float64 or tuple(out.shape) != shape or not out.is_cuda
              or not out.is_contiguous()):
            raise ValueError(f"out must be a contiguous float64 device tensor of shape {shape}")
        _check(lib().aim_rcs_noalloc(self._h, nrhs, c_void_p(x.data_ptr()), theta.numel(),
                                     c_void_p(theta.data_ptr()), phi.numel(),
                                     c_void_p(phi.data_ptr()), c_void_p(out.data_ptr()),
                                     self._stream(stream)))
        return out

    def export(self, mesh: int, what: int):
        inf = self._info
        n, nnz = inf["n"][mesh], inf["nnz"][mesh]
        K = (inf["order"] + 1) ** 3
        pad = inf["pad"][mesh]
        if what == AIM_DATA_LAMBDA64:
            out = np.zeros((n, 4, K), dtype=np.float64)
        elif what == AIM_DATA_NEAR64:
            out = np.zeros(nnz, dtype=np.complex128)
        elif what == AIM_DATA_ZDIAG64:
            out = np.zeros(n, dtype=np.complex128)
        elif what == AIM_DATA_GHAT64:
            out = np.zeros(tuple(p // 2 + 1 for p in pad), dtype=np.complex128)
        elif what == AIM_DATA_CURL64:
            out = np.zeros((n, 3, K), dtype=np.float64)
        else:
            raise ValueError(what)
        _check(lib().aim_export(self._h, mesh, what, c_void_p(out.ctypes.data), out.nbytes))
        return out

    def far_stage(self, mesh: int, x, stage: int, precision=AIM_FP64, stream=None):
        """Grid buffer after `stage` (1 projection .. 6 inverse z pass) for x
        (nrhs, n_total)."""
        torch = self._torch
        inf = self._info
        Nx, Ny, Nz = inf["grid"][mesh]
        Px, Py, Pz = inf["pad"][mesh]
        shapes = {1: (Nx, Ny, Nz), 2: (Nx, Ny, Pz), 3: (Nx, Py, Pz), 4: (Nx, Py, Pz),
                  5: (Nx, Ny, Pz), 6: (Nx, Ny, Nz)}
        dt = torch.complex128 if precision == AIM_FP64 else torch.complex64
        xx = x.reshape(-1, self.n_total).to(dt).contiguous()
        R = xx.shape[0]
        out = torch.empty((R, 4) + shapes[stage], dtype=dt, device="cuda")
        _check(lib().aim_debug_far_stage(self._h, precision, mesh, R, c_void_p(xx.data_ptr()), stage,
                                         c_void_p(out.data_ptr()), self._stream(stream)))
        return out

    def product_stage(self, mesh: int, x, stage: int, precision=AIM_FP64, stream=None):
        """The grid the product's own (pruned / in-plane) passes leave after
        `stage`, in the plain layout (nrhs, 4, A, Z) of aim_debug_product_stage;
        only the elements that header names are defined."""
        torch = self._torch
        inf = self._info
        Nx, Ny, Nz = inf["grid"][mesh]
        Px, Py, Pz = inf["pad"][mesh]
        if inf["planar_z"][mesh] >= 0:
            shapes = {1: (Nx, Ny), 3: (Nx, Py), 4: (Nx, Py), 6: (Nx, Ny)}
        else:
            shapes = {1: (Nx * Ny, Nz), 2: (Nx * Ny, Pz), 3: (Nx * Py, Pz), 4: (Nx * Py, Pz),
                      5: (Nx * Ny, Pz), 6: (Nx * Ny, Nz)}
        if stage not in shapes:
            raise ValueError(f"the product has no stage {stage} for mesh {mesh}")
        dt = torch.complex128 if precision == AIM_FP64 else torch.complex64
        xx = x.reshape(-1, self.n_total).to(dt).contiguous()
        R = xx.shape[0]
        out = torch.empty((R, 4) + shapes[stage], dtype=dt, device="cuda")
        _check(lib().aim_debug_product_stage(self._h, precision, mesh, R, c_void_p(xx.data_ptr()),
                                             stage, c_void_p(out.data_ptr()),
                                             self._stream(stream)))
        return out
