"""rsai_spmv_noalloc: the allocation-free variant of rsai_spmv, called through the C
ABI, equals rsai_spmv bit for bit on two calls in a row (the second on a smaller
matrix, so a stale work area would show) and allocates nothing."""
import ctypes

import numpy as np
import pytest

from paper_1503_04500_amd import gen

pytestmark = pytest.mark.gpu


def _call(lib, rsai, A, x, y, transpose):
    v = A.view()
    st = lib.rsai_spmv_noalloc(ctypes.byref(v), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                               1 if transpose else 0, rsai._stream())
    return st


@pytest.mark.parametrize("transpose", [False, True])
def test_noalloc_equals_spmv_on_two_calls(transpose):
    import torch
    import paper_1503_04500_amd.rsai as rsai
    lib = rsai.load()
    rsai._use_torch_allocator()
    mats = [gen.cd2d(512), gen.powerlaw(3000, seed=5)]   # second call: much smaller
    for H in mats:
        A = rsai.Matrix.from_host(H, "cuda:0")
        rng = np.random.default_rng(H.n)
        x = torch.from_numpy(rng.standard_normal(H.n)).to("cuda:0")
        ref = rsai.spmv(A, x, transpose=transpose)
        y = torch.full((H.n,), float("nan"), dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        st = _call(lib, rsai, A, x, y, transpose)
        torch.cuda.synchronize()
        after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        assert st == 0, lib.rsai_last_error()
        assert after == before, "the no-allocation entry point allocated"
        yn, rn = y.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(yn, rn), (H.name, np.max(np.abs(yn - rn)))
        # and the product itself is right (host check, fixed order not required)
        want = (H.to_dense().T if H.n <= 4000 else None)
        if want is not None:
            xv = x.cpu().numpy()
            exp = (want @ xv) if transpose else (H.to_dense() @ xv)
            assert np.allclose(yn, exp, rtol=1e-13, atol=1e-13)
        else:
            exp = H.matvec(x.cpu().numpy()) if not transpose else None
            if exp is not None:
                assert np.allclose(yn, exp, rtol=1e-13, atol=1e-13)


def test_noalloc_rejects_too_large_and_keeps_working():
    import torch
    import paper_1503_04500_amd.rsai as rsai
    lib = rsai.load()
    H = gen.cd2d(64)
    A = rsai.Matrix.from_host(H, "cuda:0")
    x = torch.ones(H.n, dtype=torch.float64, device="cuda:0")
    y = torch.zeros(H.n, dtype=torch.float64, device="cuda:0")
    # a view claiming 10^7 columns: rejected on the host before any work is queued
    big = rsai.CSCView(10_000_000, 70_000_000, A.colptr.data_ptr(), A.rowidx.data_ptr(), A.val.data_ptr())
    st = lib.rsai_spmv_noalloc(ctypes.byref(big), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0,
                               rsai._stream())
    assert st == -1 and b"work area" in lib.rsai_last_error()
    st = _call(lib, rsai, A, x, y, False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.allclose(y.cpu().numpy(), H.matvec(np.ones(H.n)), rtol=1e-14, atol=1e-14)
