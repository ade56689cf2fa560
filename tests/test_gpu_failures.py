"""Failure paths of the C ABI on the GPU: an allocator that runs out of
memory part-way through set-up makes aim_setup return AIM_ERR_NOMEM with
*out == NULL, and every block it obtained is returned (no leak)."""

import ctypes
import sys

import pytest

from workloads import sphere_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


class FailingAllocator:
    """torch caching-allocator memory for the first `budget` requests, then
    NULL; records what is live."""

    def __init__(self, budget):
        from paper_1010_1456_amd import aim as A

        self.budget = budget
        self.calls = 0
        self.live = set()
        self.freed_unknown = 0

        def _alloc(ctx, nbytes, stream):
            self.calls += 1
            if self.calls > self.budget:
                return None
            p = int(torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0)))
            self.live.add(p)
            return p

        def _free(ctx, ptr, stream):
            if ptr in self.live:
                self.live.remove(ptr)
            else:
                self.freed_unknown += 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self._a = A.ALLOC_FN(_alloc)
        self._f = A.FREE_FN(_free)
        self.struct = A.AimAllocator(None, self._a, self._f)


def _setup(fa):
    from paper_1010_1456_amd import aim as A

    m = sphere_mesh(0.5, 0.3e9, nf=4)
    keep = []
    arr = (A.AimMesh * 1)()
    arr[0] = A._mesh_struct(m.verts, m.tris, m.freq_hz, keep)
    p = A._params(0.1, 2, 0.3)
    out = ctypes.c_void_p(12345)
    st = A.lib().aim_setup(arr, 1, ctypes.byref(p), ctypes.byref(fa.struct),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                           ctypes.byref(out))
    torch.cuda.synchronize()
    return st, out


_total = {}


def _requests_of_a_full_setup():
    """Device allocations a successful set-up makes (then destroyed)."""
    from paper_1010_1456_amd import aim as A

    if "n" not in _total:
        torch.cuda.set_device(0)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        fa = FailingAllocator(10**9)
        st, out = _setup(fa)
        assert st == A.AIM_OK and out.value
        assert fa.live
        A.lib().aim_destroy(out)
        torch.cuda.synchronize()
        assert fa.live == set() and fa.freed_unknown == 0
        assert torch.cuda.memory_allocated() == before
        _total["n"] = fa.calls
    return _total["n"]


def test_setup_with_enough_memory_succeeds_and_destroy_frees_everything():
    assert _requests_of_a_full_setup() > 10


@pytest.mark.parametrize("frac", [0.0, 0.01, 0.25, 0.5, 0.75, 1.0])
def test_setup_out_of_memory_returns_nomem_and_frees_everything(frac):
    """The allocator refuses request number budget + 1 (budget = frac of what
    a full set-up needs, at most all but the last)."""
    from paper_1010_1456_amd import aim as A

    total = _requests_of_a_full_setup()
    budget = min(int(frac * total), total - 1)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    fa = FailingAllocator(budget)
    print(f"[nomem budget={budget} of {total}] aim_setup", flush=True)
    sys.stdout.flush()
    st, out = _setup(fa)
    assert st == A.AIM_ERR_NOMEM, (st, A.lib().aim_last_error())
    assert out.value is None
    assert fa.calls == budget + 1  # stopped at the first refused request
    assert fa.live == set() and fa.freed_unknown == 0
    assert torch.cuda.memory_allocated() == before
