"""GPU parity: every stage of the HIP path against the FP64 oracle.

Tolerances: FP64 path, matvec relative error <= 1e-10; FP32 (mixed) path,
<= 2e-5; operator data (projection, near-zone matrix, Green's spectrum) to
1e-12 relative to its largest entry.
"""

import math
import sys

import numpy as np
import pytest

from oracle import aim as oaim
from oracle import mom as omom
from oracle.constants import wavenumber
from oracle.rwg import build_rwg
from workloads import plate_mesh, random_current, sphere_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# name -> (mesh, stencil order M); the higher orders reach the paper's
# fifth-order reference setting (odd M puts a flat plate between grid
# planes, even M on one)
CASES = {
    "plate1": (lambda: plate_mesh(1.0, 0.3e9), 2),
    "sphere05": (lambda: sphere_mesh(0.5, 0.3e9, nf=4), 2),
    "plate2j": (lambda: plate_mesh(2.0, 0.3e9, jitter_seed=1001), 2),
    "sphere05_m3": (lambda: sphere_mesh(0.5, 0.3e9, nf=4), 3),
    "plate2j_m4": (lambda: plate_mesh(2.0, 0.3e9, jitter_seed=1001), 4),
    "plate1_m5": (lambda: plate_mesh(1.0, 0.3e9), 5),
    "sphere05_m5": (lambda: sphere_mesh(0.5, 0.3e9, nf=4), 5),
}


class Case:
    def __init__(self, name):
        from paper_1010_1456_amd import aim as A

        self.name = name
        make, self.order = CASES[name]
        self.mesh = make()
        m = self.mesh
        self.k = wavenumber(m.freq_hz)
        _log(f"[case {name}] oracle set-up (M={self.order})")
        self.rwg = build_rwg(m.verts, m.tris)
        self.op = oaim.build_operator(self.rwg, self.k, 0.1 * m.lam, self.order, 0.3 * m.lam)
        _log(f"[case {name}] GPU set-up N={self.rwg.n}")
        self.plan = A.Plan([(m.verts, m.tris, m.freq_hz)], order=self.order)
        torch.cuda.synchronize()
        info = self.plan.info()
        self.pad = info["pad"][0]
        self.ghat = oaim.green_spectrum(self.k, self.op.grid, self.pad)


_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = Case(name)
    return _cache[name]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def rel_max(a, b):
    """Element-wise: max |a - b| / max |b|."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("name", list(CASES))
def test_projection_weights(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    lam = c.plan.export(0, A.AIM_DATA_LAMBDA64)
    assert np.abs(lam - c.op.lam).max() <= 1e-13 * np.abs(c.op.lam).max()


@pytest.mark.parametrize("name", list(CASES))
def test_near_matrix_and_diagonal(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    near = c.plan.export(0, A.AIM_DATA_NEAR64)
    ref = c.op.near.data
    assert np.abs(near - ref).max() <= 1e-12 * np.abs(ref).max()
    zd = c.plan.export(0, A.AIM_DATA_ZDIAG64)
    assert np.abs(zd - c.op.zmom_diag).max() <= 1e-12 * np.abs(c.op.zmom_diag).max()


@pytest.mark.parametrize("name", list(CASES))
def test_green_spectrum_octant(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    g = c.plan.export(0, A.AIM_DATA_GHAT64)
    Px, Py, Pz = c.pad
    ref = c.ghat[: Px // 2 + 1, : Py // 2 + 1, : Pz // 2 + 1] / (Px * Py * Pz)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_far_stages(name, prec):
    """Each pass of the propagation step against numpy FFTs of the oracle's
    projected grids (pruned shapes, unnormalised inverses)."""
    from paper_1010_1456_amd import aim as A

    c = case(name)
    P = A.AIM_FP64 if prec == "fp64" else A.AIM_MIXED
    tol = 1e-12 if prec == "fp64" else 3e-6
    x = random_current(c.rwg.n, nrhs=2, seed=3)
    Nx, Ny, Nz = (int(v) for v in c.op.grid.n)
    Px, Py, Pz = c.pad
    s = oaim.anterpolate(c.op, x).reshape(2, 4, Nx, Ny, Nz)
    st2 = np.fft.fft(s, n=Pz, axis=4)
    st3 = np.fft.fft(st2, n=Py, axis=3)
    full = np.fft.fft(st3, n=Px, axis=2) * (c.ghat / (Px * Py * Pz))[None, None]
    st4 = (np.fft.ifft(full, axis=2) * Px)[:, :, :Nx]
    st5 = (np.fft.ifft(st4, axis=3) * Py)[:, :, :, :Ny]
    st6 = (np.fft.ifft(st5, axis=4) * Pz)[..., :Nz]
    refs = {1: s, 2: st2, 3: st3, 4: st4, 5: st5, 6: st6}
    xt = torch.from_numpy(x).cuda()
    for stage in range(1, 7):
        _log(f"[far_stages {name} {prec}] stage {stage}")
        got = c.plan.far_stage(0, xt, stage, P).cpu().numpy()
        r = refs[stage]
        err = np.abs(got - r).max() / np.abs(r).max()
        assert err <= tol, (stage, err)


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_fp64(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    x = random_current(c.rwg.n, nrhs=3, seed=7)
    ref = oaim.matvec_fft(c.op, x)
    y = c.plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    for r in range(3):
        assert rel(y[r], ref[r]) <= 1e-10
        assert rel_max(y[r], ref[r]) <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_mixed(name):
    from paper_1010_1456_amd import aim as A

    c = case(name)
    x = random_current(c.rwg.n, nrhs=2, seed=8)
    ref = oaim.matvec_fft(c.op, x)
    xt = torch.from_numpy(x.astype(np.complex64)).cuda()
    y = c.plan.matvec(xt, A.AIM_MIXED).cpu().numpy().astype(np.complex128)
    ref32 = oaim.matvec_fft(c.op, x.astype(np.complex64).astype(np.complex128))
    for r in range(2):
        assert rel(y[r], ref32[r]) <= 2e-5
        assert rel_max(y[r], ref32[r]) <= 2e-5
    assert rel(y, ref) <= 1e-4
    # the solver's form: the same c64 arithmetic on c128 vectors, narrowed as
    # x is read and widened as y is written, so equal to the c64 product bit
    # for bit
    x64 = x.astype(np.complex64).astype(np.complex128)
    y_io = c.plan.matvec(torch.from_numpy(x64).cuda(), A.AIM_MIXED_IO64).cpu().numpy()
    assert np.array_equal(y_io, y)
    for r in range(2):
        assert rel_max(y_io[r], ref32[r]) <= 2e-5


@pytest.mark.parametrize("name,plane", [("plate1", 1), ("plate2j_m4", 2), ("plate1_m5", -1),
                                        ("sphere05", -1)])
def test_planar_detection(name, plane):
    """A flat plate takes the in-plane propagation when every projection
    weight falls on one grid plane: even M puts it on the middle plane, odd M
    between two planes (weights on all M + 1 planes)."""
    c = case(name)
    assert c.plan.info()["planar_z"][0] == plane
    if plane >= 0:
        nodes = oaim._node_index(c.op.grid, c.op.anc) % int(c.op.grid.n[2])
        assert np.all(np.where(np.abs(c.op.lam).max(axis=1) > 0, nodes == plane, True))


def test_setup_phase_times():
    """Every set-up phase is timed; the near-zone fill and the host plan take
    measurable time, and together the phases stay within the plan's wall time."""
    import time

    from paper_1010_1456_amd import aim as A

    m = CASES["sphere05"][0]()
    t0 = time.perf_counter()
    plan = A.Plan([(m.verts, m.tris, m.freq_hz)])
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    t = plan.info()["setup_ms"][0]
    assert tuple(t) == A.SETUP_PHASES
    assert all(v >= 0 for v in t.values())
    assert t["host_plan"] > 0 and t["near_fill"] > 0 and t["projection"] > 0
    assert sum(t.values()) <= wall_ms
    plan.close()


def test_matvec_direct_sum_agrees():
    """The GPU product equals the plain direct-summation definition."""
    from paper_1010_1456_amd import aim as A

    c = case("sphere05")
    x = random_current(c.rwg.n, nrhs=1, seed=9)[0]
    ref = oaim.matvec_direct(c.op, x)
    y = c.plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    assert rel(y, ref) <= 1e-10


def _strip_mesh(length_lambda, width_lambda, freq_hz, per_lambda=9):
    """Structured rectangular plate in z = 0 (squares split along the
    (i, j)-(i+1, j+1) diagonal, counter-clockwise about +z)."""
    from workloads.meshes import wavelength

    lam = wavelength(freq_hz)
    nx, ny = round(length_lambda * per_lambda), round(width_lambda * per_lambda)
    xs = (np.arange(nx + 1) / per_lambda - length_lambda / 2) * lam
    ys = (np.arange(ny + 1) / per_lambda - width_lambda / 2) * lam
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    vid = lambda i, j: i * (ny + 1) + j  # noqa: E731
    tris = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris += [(a, b, c), (a, c, d)]
    return verts, np.asarray(tris, dtype=np.int32)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_far_stages_long_x_lines(prec):
    """A 40 x 0.5 lambda strip: a three-stage x FFT (864 points) with few lines
    per x-pass work-group (4 for c64, 2 for c128) in the thin layout. Every
    pass against numpy FFTs of the oracle's projected grid."""
    from paper_1010_1456_amd import aim as A

    freq = 0.3e9
    verts, tris = _strip_mesh(40.0, 0.5, freq)
    k = wavenumber(freq)
    lam_m = 299_792_458.0 / freq
    rwg = build_rwg(verts, tris)
    grid = oaim.grid_plan(rwg.verts, 0.1 * lam_m, 2)
    anc = oaim.anchors(grid, rwg.centre)
    op = oaim.AIMOperator(rwg=rwg, k=k, grid=grid, anc=anc, lam=oaim.projection(rwg, grid, anc),
                          near=None, zmom_diag=None)
    plan = A.Plan([(verts, tris, freq)])
    Px, Py, Pz = plan.info()["pad"][0]
    assert Px >= 769  # at most 4 (c64) / 2 (c128) lines per x-pass work-group
    ghat = oaim.green_spectrum(k, grid, (Px, Py, Pz))
    P = A.AIM_FP64 if prec == "fp64" else A.AIM_MIXED
    tol = 1e-12 if prec == "fp64" else 3e-6
    x = random_current(rwg.n, nrhs=2, seed=11)
    Nx, Ny, Nz = (int(v) for v in grid.n)
    s = oaim.anterpolate(op, x).reshape(2, 4, Nx, Ny, Nz)
    st2 = np.fft.fft(s, n=Pz, axis=4)
    st3 = np.fft.fft(st2, n=Py, axis=3)
    full = np.fft.fft(st3, n=Px, axis=2) * (ghat / (Px * Py * Pz))[None, None]
    st4 = (np.fft.ifft(full, axis=2) * Px)[:, :, :Nx]
    st5 = (np.fft.ifft(st4, axis=3) * Py)[:, :, :, :Ny]
    st6 = (np.fft.ifft(st5, axis=4) * Pz)[..., :Nz]
    refs = {1: s, 2: st2, 3: st3, 4: st4, 5: st5, 6: st6}
    xt = torch.from_numpy(x).cuda()
    for stage in range(1, 7):
        _log(f"[far_stages strip {prec}] stage {stage}")
        got = plan.far_stage(0, xt, stage, P).cpu().numpy()
        r = refs[stage]
        err = np.abs(got - r).max() / np.abs(r).max()
        assert err <= tol, (stage, err)
    plan.close()


@pytest.mark.parametrize("name", ["sphere05", "plate2j"])
def test_products_with_changing_right_hand_side_counts(name):
    """One plan, products with 4, 1, 3 and 1 right-hand sides in turn, both
    precisions: the persistent source and forward-z grids (zero where nothing
    is written) and the interleaved field grid keep every product exact."""
    from paper_1010_1456_amd import aim as A

    c = case(name)
    for r, seed in ((4, 51), (1, 52), (3, 53), (1, 54)):
        x = random_current(c.rwg.n, nrhs=r, seed=seed)
        ref = oaim.matvec_fft(c.op, x)
        y = c.plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
        y32 = c.plan.matvec(torch.from_numpy(x).cuda(), A.AIM_MIXED_IO64).cpu().numpy()
        ref32 = oaim.matvec_fft(c.op, x.astype(np.complex64).astype(np.complex128))
        for k in range(r):
            assert rel(y[k], ref[k]) <= 1e-10, (r, k)
            assert rel_max(y32[k], ref32[k]) <= 2e-5, (r, k)


def _reference_stages(c, x):
    """The propagation step's grids from the oracle's projected sources:
    numpy FFTs on the padded grid, the spectrum scaled by 1/(Px Py Pz),
    unnormalised inverses (as the library keeps them)."""
    R = x.shape[0]
    Nx, Ny, Nz = (int(v) for v in c.op.grid.n)
    Px, Py, Pz = c.pad
    s = oaim.anterpolate(c.op, x).reshape(R, 4, Nx, Ny, Nz)
    st2 = np.fft.fft(s, n=Pz, axis=4)
    st3 = np.fft.fft(st2, n=Py, axis=3)
    full = np.fft.fft(st3, n=Px, axis=2) * (c.ghat / (Px * Py * Pz))[None, None]
    st4 = (np.fft.ifft(full, axis=2) * Px)[:, :, :Nx]
    st5 = (np.fft.ifft(st4, axis=3) * Py)[:, :, :, :Ny]
    st6 = (np.fft.ifft(st5, axis=4) * Pz)[..., :Nz]
    return {1: s, 2: st2, 3: st3, 4: st4, 5: st5, 6: st6}


def _occupancy(c):
    """Occupied grid nodes (a non-zero projection weight of some basis), as a
    boolean (Nx, Ny, Nz) array, from the oracle's projection."""
    Nx, Ny, Nz = (int(v) for v in c.op.grid.n)
    idx = oaim._node_index(c.op.grid, c.op.anc)  # (N, K)
    hit = np.abs(c.op.lam).max(axis=1) > 0  # (N, K)
    occ = np.zeros(Nx * Ny * Nz, dtype=bool)
    occ[idx[hit]] = True
    return occ.reshape(Nx, Ny, Nz)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_product_stages(name, prec):
    """The product's own passes (pruned to the occupied nodes, lines and
    rows; in-plane for a scatterer on one grid plane), each stage against
    numpy FFTs of the oracle's projected grids, over the elements the next
    step reads (see aim_debug_product_stage)."""
    from paper_1010_1456_amd import aim as A

    c = case(name)
    P = A.AIM_FP64 if prec == "fp64" else A.AIM_MIXED
    tol = 1e-12 if prec == "fp64" else 3e-6
    x = random_current(c.rwg.n, nrhs=2, seed=13)
    refs = _reference_stages(c, x)
    Nx, Ny, Nz = (int(v) for v in c.op.grid.n)
    Px, Py, Pz = c.pad
    xt = torch.from_numpy(x).cuda()
    zp = c.plan.info()["planar_z"][0]
    occ = _occupancy(c)
    if zp >= 0:  # in-plane path: stages 1, 3, 4, 6 on the plane z = zp
        assert not occ[:, :, np.arange(Nz) != zp].any()
        sp = refs[1][..., zp]
        # the 2-D spectrum of g(x, y, 0): the 3-D spectrum summed over kz, / Pz
        g2 = c.ghat.sum(axis=2) / Pz
        st3p = np.fft.fft(sp, n=Py, axis=3)
        st4p = (np.fft.ifft(np.fft.fft(st3p, n=Px, axis=2) * (g2 / (Px * Py))[None, None],
                            axis=2) * Px)[:, :, :Nx]
        plane_refs = {1: sp, 3: st3p, 4: st4p, 6: refs[6][..., zp]}
        for stage, r in plane_refs.items():
            _log(f"[product_stages {name} {prec}] plane stage {stage}")
            got = c.plan.product_stage(0, xt, stage, P).cpu().numpy()
            err = np.abs(got - r).max() / np.abs(r).max()
            assert err <= tol, (stage, err)
        for stage in (2, 5):
            with pytest.raises(ValueError):
                c.plan.product_stage(0, xt, stage, P)
        return
    lines = occ.any(axis=2)  # (Nx, Ny) occupied z lines
    ymask = np.zeros((Nx, Ny), dtype=bool)  # rows inside each x plane's occupied y range
    for i in range(Nx):
        ys = np.flatnonzero(lines[i])
        if ys.size:
            ymask[i, ys[0]:ys[-1] + 1] = True
    # occupied lines over their occupied z range, less the longest run of
    # unoccupied nodes inside it (the first on ties): the nodes the inverse z
    # pass writes, every occupied node among them
    zmask = np.zeros((Nx, Ny, Nz), dtype=bool)
    for i, j in zip(*np.nonzero(lines)):
        zs = np.flatnonzero(occ[i, j])
        zmask[i, j, zs[0]:zs[-1] + 1] = True
        if zs.size > 1:
            k = int(np.argmax(np.diff(zs)))
            zmask[i, j, zs[k] + 1:zs[k + 1]] = False
    assert zmask[occ].all()
    R = x.shape[0]
    for stage in range(1, 7):
        _log(f"[product_stages {name} {prec}] stage {stage}")
        got = c.plan.product_stage(0, xt, stage, P).cpu().numpy()
        r = refs[stage].reshape(got.shape)
        if stage == 5:
            m = np.broadcast_to(ymask.reshape(1, 1, Nx * Ny, 1), got.shape)
        elif stage == 6:
            m = np.broadcast_to(zmask.reshape(1, 1, Nx * Ny, Nz), got.shape)
        else:
            m = np.ones(got.shape, dtype=bool)
        assert m.any()
        err = np.abs(got[m] - r[m]).max() / np.abs(r[m]).max()
        assert err <= tol, (stage, err)
    assert R == 2


def test_inspection_after_product_on_a_plate():
    """A product on the in-plane path with three right-hand sides, then the
    full 3-D inspection with one on the same plan: the source grid written in
    the plane layout is cleared before the 3-D layout uses it, so every
    inspected stage is exact."""
    from paper_1010_1456_amd import aim as A

    c = case("plate2j")
    assert c.plan.info()["planar_z"][0] >= 0
    x3 = torch.from_numpy(random_current(c.rwg.n, nrhs=3, seed=61)).cuda()
    c.plan.matvec(x3, A.AIM_FP64)
    c.plan.matvec(x3.to(torch.complex64), A.AIM_MIXED)
    x = random_current(c.rwg.n, nrhs=1, seed=62)
    refs = _reference_stages(c, x)
    xt = torch.from_numpy(x).cuda()
    for P, tol in ((A.AIM_FP64, 1e-12), (A.AIM_MIXED, 3e-6)):
        for stage in range(1, 7):
            got = c.plan.far_stage(0, xt, stage, P).cpu().numpy()
            r = refs[stage]
            assert np.abs(got - r).max() <= tol * np.abs(r).max(), (P, stage)


def _l_plate(freq_hz):
    """A 2-lambda plate with one quadrant (x > 0, y > 0) removed: a flat
    scatterer on one grid plane whose plane holds nodes with no stencil
    entries inside its bounding box."""
    m = plate_mesh(2.0, freq_hz, jitter_seed=77)
    cen = m.verts[m.tris].mean(axis=1)
    keep = ~((cen[:, 0] > 0) & (cen[:, 1] > 0))
    tris = m.tris[keep]
    used = np.unique(tris)
    remap = np.full(m.verts.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return m.verts[used], remap[tris].astype(np.int32)


def test_product_after_inspection_on_an_l_shaped_plate():
    """Inspection (full 3-D passes) first, then products on the in-plane path
    of a non-rectangular plate: no stale source values reach the product."""
    from paper_1010_1456_amd import aim as A

    freq = 0.3e9
    verts, tris = _l_plate(freq)
    lam = 299_792_458.0 / freq
    k = wavenumber(freq)
    rwg = build_rwg(verts, tris)
    op = oaim.build_operator(rwg, k, 0.1 * lam, 2, 0.3 * lam)
    plan = A.Plan([(verts, tris, freq)])
    assert plan.info()["planar_z"][0] >= 0
    xi = torch.from_numpy(random_current(rwg.n, nrhs=2, seed=71)).cuda()
    for P in (A.AIM_FP64, A.AIM_MIXED):
        for stage in (1, 6):
            plan.far_stage(0, xi, stage, P)
    x = random_current(rwg.n, nrhs=2, seed=72)
    ref = oaim.matvec_fft(op, x)
    y = plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    y32 = plan.matvec(torch.from_numpy(x).cuda(), A.AIM_MIXED_IO64).cpu().numpy()
    ref32 = oaim.matvec_fft(op, x.astype(np.complex64).astype(np.complex128))
    for r in range(2):
        assert rel_max(y[r], ref[r]) <= 1e-10
        assert rel_max(y32[r], ref32[r]) <= 2e-5
    plan.close()


# Spheres whose FFT lengths have pipelined y / x / y kernels: 72 = 9 x 8 (odd
# first radix, even last), 81 = 9 x 9 (no pruned stage), 144 = 12 x 12 (both
# pruned), meshed coarsely so that the oracle's operator builds in seconds.
PIPE_CASES = {
    "sphere165": (lambda: sphere_mesh(1.65, 0.3e9, nf=10), 72),
    "sphere2": (lambda: sphere_mesh(2.0, 0.3e9, nf=8), 81),
    "sphere355": (lambda: sphere_mesh(3.55, 0.3e9, nf=14), 144),
}
_pipe_ops = {}


def _pipe_case(name):
    if name not in _pipe_ops:
        m = PIPE_CASES[name][0]()
        k = wavenumber(m.freq_hz)
        rwg = build_rwg(m.verts, m.tris)
        _log(f"[pipeline {name}] oracle set-up N={rwg.n}")
        op = oaim.build_operator(rwg, k, 0.1 * m.lam, 2, 0.3 * m.lam)
        _pipe_ops[name] = (m, rwg, op)
    return _pipe_ops[name]


@pytest.mark.parametrize("name", list(PIPE_CASES))
@pytest.mark.parametrize("groups", [2, 4])
def test_pipelined_passes(name, groups):
    """The forward y, x and inverse y passes pipelined over field groups (one
    launch holding the x pass of one group beside the y passes of others):
    products with 1 and 3 right-hand sides against the oracle, both paths,
    and the grids the pipeline leaves (x pass, inverse y pass) against numpy
    FFTs of the oracle's projected grids."""
    from paper_1010_1456_amd import aim as A

    m, rwg, op = _pipe_case(name)
    plan = A.Plan([(m.verts, m.tris, m.freq_hz)], xy_groups=groups)
    inf = plan.info()
    assert inf["pad"][0][0] == PIPE_CASES[name][1] == inf["pad"][0][1]
    assert inf["xy_groups"][0] == (groups, groups)
    for nrhs, seed in ((1, 81), (3, 82)):
        x = random_current(rwg.n, nrhs=nrhs, seed=seed)
        ref = oaim.matvec_fft(op, x)
        y = plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
        x32 = x.astype(np.complex64)
        ref32 = oaim.matvec_fft(op, x32.astype(np.complex128))
        y32 = plan.matvec(torch.from_numpy(x32).cuda(), A.AIM_MIXED).cpu().numpy()
        for r in range(nrhs):
            assert rel_max(y[r], ref[r]) <= 1e-10, (nrhs, r)
            assert rel(y32[r], ref32[r]) <= 2e-5, (nrhs, r)
            assert rel_max(y32[r], ref32[r]) <= 2e-5, (nrhs, r)
    # the pipeline's own grids
    c = type("C", (), {})()
    c.op, c.k, c.pad = op, wavenumber(m.freq_hz), inf["pad"][0]
    c.ghat = oaim.green_spectrum(c.k, op.grid, c.pad)
    x = random_current(rwg.n, nrhs=2, seed=83)
    refs = _reference_stages(c, x)
    xt = torch.from_numpy(x).cuda()
    Nx, Ny, Nz = (int(v) for v in op.grid.n)
    occ = _occupancy(c)
    lines = occ.any(axis=2)
    ymask = np.zeros((Nx, Ny), dtype=bool)
    for i in range(Nx):
        ys = np.flatnonzero(lines[i])
        if ys.size:
            ymask[i, ys[0]:ys[-1] + 1] = True
    for P, tol in ((A.AIM_FP64, 1e-12), (A.AIM_MIXED, 3e-6)):
        for stage in (4, 5):
            got = plan.product_stage(0, xt, stage, P).cpu().numpy()
            r = refs[stage].reshape(got.shape)
            msk = (np.ones(got.shape, dtype=bool) if stage == 4
                   else np.broadcast_to(ymask.reshape(1, 1, Nx * Ny, 1), got.shape))
            err = np.abs(got[msk] - r[msk]).max() / np.abs(r[msk]).max()
            assert err <= tol, (P, stage, err)
    plan.close()


def test_pipeline_group_count_is_validated():
    from paper_1010_1456_amd import aim as A

    m = plate_mesh(1.0, 0.3e9)
    with pytest.raises(A.AimError):
        A.Plan([(m.verts, m.tris, m.freq_hz)], xy_groups=3)


@pytest.mark.parametrize("name", list(CASES))
def test_64_byte_tile_rows(name):
    """The x and strided y passes with 64-byte tile rows (half the lines per
    work-group): products against the oracle and every pass against numpy
    FFTs of the oracle's projected grids (3-D, thin and in-plane layouts)."""
    from paper_1010_1456_amd import aim as A

    c = case(name)
    plan = A.Plan([(c.mesh.verts, c.mesh.tris, c.mesh.freq_hz)], order=c.order, tile_rows=64)
    assert plan.info()["tile_bytes"][0] == ((64, 64), (64, 64))
    for nrhs, seed in ((1, 111), (3, 112)):
        x = random_current(c.rwg.n, nrhs=nrhs, seed=seed)
        ref = oaim.matvec_fft(c.op, x)
        xt = torch.from_numpy(x).cuda()
        y = plan.matvec(xt, A.AIM_FP64).cpu().numpy()
        x32 = x.astype(np.complex64)
        ref32 = oaim.matvec_fft(c.op, x32.astype(np.complex128))
        y32 = plan.matvec(torch.from_numpy(x32).cuda(), A.AIM_MIXED).cpu().numpy()
        for r in range(nrhs):
            assert rel_max(y[r], ref[r]) <= 1e-10, (nrhs, r)
            assert rel_max(y32[r], ref32[r]) <= 2e-5, (nrhs, r)
    x = random_current(c.rwg.n, nrhs=2, seed=113)
    xt = torch.from_numpy(x).cuda()
    refs = _reference_stages(c, x)
    for P, tol in ((A.AIM_FP64, 1e-12), (A.AIM_MIXED, 3e-6)):
        for stage in range(1, 7):
            got = plan.far_stage(0, xt, stage, P).cpu().numpy()
            assert np.abs(got - refs[stage]).max() <= tol * np.abs(refs[stage]).max(), (P, stage)
    plan.close()


def test_tuning_values_are_validated():
    from paper_1010_1456_amd import aim as A

    m = plate_mesh(1.0, 0.3e9)
    p = A._params(0.1, 2, 0.3)
    p.tuning = 3 << 8
    L = A.lib()
    keep = []
    arr = (A.AimMesh * 1)()
    arr[0] = A._mesh_struct(m.verts, m.tris, m.freq_hz, keep)
    import ctypes

    h = ctypes.c_void_p()
    assert L.aim_setup(arr, 1, ctypes.byref(p), None, None, ctypes.byref(h)) == A.AIM_ERR_ARG
    assert h.value is None
    for bad in (65 << 16, 1 << 24):  # tuning right-hand sides above 64; unused bits
        p.tuning = bad
        assert L.aim_setup(arr, 1, ctypes.byref(p), None, None, ctypes.byref(h)) == A.AIM_ERR_ARG
        assert h.value is None


def test_tuning_with_several_right_hand_sides():
    """Set-up timing its variants on 4 right-hand sides per mesh: the chosen
    variants' products of 4 right-hand sides against the oracle."""
    from paper_1010_1456_amd import aim as A

    c = case("sphere05")
    plan = A.Plan([(c.mesh.verts, c.mesh.tris, c.mesh.freq_hz)], order=c.order, tune_rhs=4)
    x = random_current(c.rwg.n, nrhs=4, seed=114)
    ref = oaim.matvec_fft(c.op, x)
    y = plan.matvec(torch.from_numpy(x).cuda(), A.AIM_FP64).cpu().numpy()
    x32 = x.astype(np.complex64)
    ref32 = oaim.matvec_fft(c.op, x32.astype(np.complex128))
    y32 = plan.matvec(torch.from_numpy(x32).cuda(), A.AIM_MIXED).cpu().numpy()
    for r in range(4):
        assert rel_max(y[r], ref[r]) <= 1e-10, r
        assert rel_max(y32[r], ref32[r]) <= 2e-5, r
    plan.close()
