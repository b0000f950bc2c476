"""Allocator-failure injection through rsai_set_allocator: an allocation that fails
at any point of a build, a solve or an adjoint gives RSAI_E_NOMEM and leaves no
device memory behind; the library keeps working afterwards."""
import ctypes

import numpy as np
import pytest

from paper_1503_04500_amd import gen

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """Wraps torch's caching allocator; fails the fail_at-th request (1-based)."""

    def __init__(self):
        import torch
        import paper_1503_04500_amd.rsai as rsai
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_at = 0
        self._a = rsai._ALLOC_T(self.alloc)
        self._f = rsai._FREE_T(self.free)

    def alloc(self, size, stream, ctx):
        self.calls += 1
        if self.fail_at and self.calls == self.fail_at:
            return None
        p = self.torch.cuda.caching_allocator_alloc(int(size), self.torch.cuda.current_device(), stream or 0)
        self.live[p] = int(size)
        return p

    def free(self, ptr, stream, ctx):
        if ptr:
            assert ptr in self.live, "free of a pointer the allocator did not hand out"
            del self.live[ptr]
            self.torch.cuda.caching_allocator_delete(ptr)

    def install(self):
        import paper_1503_04500_amd.rsai as rsai
        lib = rsai.load()
        assert lib.rsai_set_allocator(ctypes.cast(self._a, ctypes.c_void_p), ctypes.cast(self._f, ctypes.c_void_p),
                                      None) == 0

    def reset(self, fail_at=0):
        self.calls = 0
        self.fail_at = fail_at


@pytest.fixture
def counting(monkeypatch):
    import paper_1503_04500_amd.rsai as rsai
    real = rsai._use_torch_allocator
    # the binding re-installs torch's allocator on every build: keep ours in place
    monkeypatch.setattr(rsai, "_use_torch_allocator", lambda: None)
    c = CountingAllocator()
    c.install()
    yield c
    monkeypatch.undo()
    real()


def _sweep(counting, run, label):
    """Count the allocations of run() (after one warm-up call), then fail each one in
    turn. run() releases everything it allocates, on success and on failure."""
    import paper_1503_04500_amd.rsai as rsai
    run()
    counting.torch.cuda.synchronize()
    base = set(counting.live)
    counting.reset()
    run()
    total = counting.calls
    assert total >= 1, label
    for k in range(1, total + 1):
        counting.reset(fail_at=k)
        with pytest.raises(rsai.RSAIError) as ei:
            run()
        assert ei.value.code == -4, (label, k, ei.value)
        counting.torch.cuda.synchronize()
        assert set(counting.live) == base, (label, k, "leaked", len(counting.live) - len(base))
    counting.reset()
    return total


def _build_run(A, **kw):
    import paper_1503_04500_amd.rsai as rsai

    def run():
        p = rsai.build(A, **kw)
        try:
            p.nnz()
        finally:
            p.close()
    return run


def test_build_failures_leave_nothing(counting):
    import paper_1503_04500_amd.rsai as rsai
    A = rsai.Matrix.from_host(gen.cd2d(40, seed=1), "cuda:0")
    _sweep(counting, _build_run(A, c=3, lmax=8, eps=0.4, tol=1e-3, keep_factors=True), "build")
    assert not counting.live


def test_batched_build_solve_adjoint_failures_leave_nothing(counting):
    import torch
    import paper_1503_04500_amd.rsai as rsai
    Hs = [gen.cd2d(24, seed=2), gen.powerlaw(1500, seed=3, lmax=20)]
    mats = [rsai.Matrix.from_host(h, "cuda:0") for h in Hs]
    kw = dict(c=3, lmax=4, eps=0.4, tol=1e-3, keep_factors=True)

    def build():
        p = rsai.build_batched(mats, **kw)
        try:
            p.nnz(0)
            p.nnz(1)
        finally:
            p.close()

    _sweep(counting, build, "batched build")

    dA = torch.zeros(Hs[1].nnz, dtype=torch.float64, device="cuda:0")

    def build_and_adjoint():
        p = rsai.build_batched(mats, **kw)
        try:
            p.backward(None, 1.0, dA, mat=1)
        finally:
            p.close()

    _sweep(counting, build_and_adjoint, "build + adjoint")

    plan = rsai.build_batched(mats, **kw)
    b = torch.ones(Hs[0].n, dtype=torch.float64, device="cuda:0")
    _sweep(counting, lambda: plan.bicgstab(b), "bicgstab")
    _sweep(counting, lambda: plan.bicgstab(b, precond=False), "bicgstab without M")
    plan.close()
    counting.torch.cuda.synchronize()
    assert not counting.live
    # the library is usable after the failures
    p = rsai.build(mats[0], c=3, lmax=8, eps=0.4, tol=1e-3)
    assert p.nnz() > 0
    p.close()
