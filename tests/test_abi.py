"""The C ABI library loads here (no GPU) and exports every function that
include/rsai.h declares; argument errors come back as status codes."""
import ctypes
import os
import re

import pytest

import paper_1503_04500_amd.rsai as rsai

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsai.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsai_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("rsai_build", "rsai_build_batched", "rsai_apply", "rsai_backward", "rsai_export_M",
                 "rsai_plan_nnz", "rsai_destroy", "rsai_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported():
    if not os.path.exists(rsai.LIB_PATH):
        pytest.skip("librsai.so not built")
    lib = ctypes.CDLL(rsai.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_default_and_tiers():
    if not os.path.exists(rsai.LIB_PATH):
        pytest.skip("librsai.so not built")
    p = rsai.params()
    assert (p.c, p.lmax, p.drop) == (3, 10, 1)
    assert abs(p.eps - 0.4) < 1e-15 and abs(p.tol - 1e-3) < 1e-15
    g0, m0, q0 = rsai.tier_info(0)
    assert g0 * (64 // g0) == 64 and q0 <= m0
    with pytest.raises(rsai.RSAIError) as ei:
        rsai.tier_info(99)
    assert ei.value.code == -1


def test_argument_errors_without_gpu():
    if not os.path.exists(rsai.LIB_PATH):
        pytest.skip("librsai.so not built")
    lib = rsai.load()
    out = ctypes.c_void_p()
    p = rsai.params()
    # NULL matrix
    assert lib.rsai_build(None, ctypes.byref(p), None, ctypes.byref(out)) == -1
    assert not out.value
    # bad c, bad lmax, bad drop mode, bad schedule
    v = rsai.CSCView(4, 4, 8, 8, 8)
    for field, val in (("c", 0), ("c", 9), ("lmax", -1), ("drop", 7), ("sched", 5), ("tier0", 9)):
        q = rsai.params()
        setattr(q, field, val)
        assert lib.rsai_build(ctypes.byref(v), ctypes.byref(q), None, ctypes.byref(out)) == -1, field
        assert b"" != lib.rsai_last_error()
    # bad sizes: nnz < n
    bad = rsai.CSCView(4, 3, 8, 8, 8)
    assert lib.rsai_build(ctypes.byref(bad), ctypes.byref(p), None, ctypes.byref(out)) == -1
    # plan queries on NULL
    n = ctypes.c_int64()
    assert lib.rsai_plan_nnz(None, 0, ctypes.byref(n)) == -1
    assert lib.rsai_destroy(None) == 0
    assert lib.rsai_set_allocator(ctypes.c_void_p(1), None, None) == -1
    assert lib.rsai_rebuild(None, 1, None) == -1
    it, rel = ctypes.c_int32(), ctypes.c_double()
    assert lib.rsai_bicgstab(None, 0, None, None, 1e-8, 10, 1, 1, ctypes.byref(it), ctypes.byref(rel), None) == -1
    assert lib.rsai_bicgstab_left(None, None, 0, None, None, 1e-8, 10, 1, ctypes.byref(it), ctypes.byref(rel),
                                  None) == -1
    assert lib.rsai_transpose(None, None, None, None, None) == -1
    tf = ctypes.c_double()
    assert lib.rsai_peak_fp64(1 << 16, None, None) == -1
    assert lib.rsai_peak_fp64(15, ctypes.byref(tf), None) == -1
    cnt, best = ctypes.c_int32(), ctypes.c_int32()
    assert lib.rsai_autotune(None, ctypes.byref(p), 1, None, None, 0, ctypes.byref(cnt), ctypes.byref(best)) == -1
    # the allocation-free SpMV checks its arguments and its work-area limit on the host
    assert lib.rsai_spmv_noalloc(None, None, None, 0, None) == -1
    huge = rsai.CSCView(10_000_000, 70_000_000, 8, 8, 8)
    assert lib.rsai_spmv_noalloc(ctypes.byref(huge), ctypes.c_void_p(8), ctypes.c_void_p(8), 0, None) == -1
    assert b"work area" in lib.rsai_last_error()
    bad = rsai.params()
    bad.route = 3
    assert lib.rsai_build(ctypes.byref(rsai.CSCView(4, 4, 8, 8, 8)), ctypes.byref(bad), None, ctypes.byref(out)) == -1
    bad = rsai.params(spill_capacity=-1)
    assert lib.rsai_build(ctypes.byref(rsai.CSCView(4, 4, 8, 8, 8)), ctypes.byref(bad), None, ctypes.byref(out)) == -1
    assert b"spill_capacity" in lib.rsai_last_error()
    assert rsai.params().spill_capacity == 0


def test_params_are_fresh_copies():
    """rsai.params reuses the struct it made for the same arguments: each call still
    returns a separate copy (changing one leaves the next call's alone), different
    arguments give different structs, and a repeated call equals a first one."""
    import paper_1503_04500_amd.rsai as rsai
    a = rsai.params(c=3, lmax=8, eps=0.4, tol=1e-3)
    a.c = 5
    a.tune_count = 3
    b = rsai.params(c=3, lmax=8, eps=0.4, tol=1e-3)
    assert b.c == 3 and b.tune_count == 0 and b.lmax == 8
    assert bytes(b) == bytes(rsai._make_params(3, 8, 0.4, "fixed", 1e-3, "batched", True, -1, False, -1, -1,
                                               False, 0, False, -1, -1, 0))
    assert rsai.params(c=4, lmax=8).c == 4 and rsai.params(c=3, lmax=8).c == 3
    assert rsai.params(drop="adaptive").drop == rsai.DROP["adaptive"]
    # the tuning array is converted once and reused while the table is the same
    arr1, n1 = rsai.tune_entries()
    arr2, n2 = rsai.tune_entries()
    assert arr1 is arr2 and n1 == n2
    arr3, n3 = rsai.tune_entries([])
    assert n3 == 0


def test_no_cpu_fallback():
    """The binding refuses host tensors instead of computing on the CPU."""
    import torch
    with pytest.raises(ValueError):
        rsai.Matrix(torch.zeros(3, dtype=torch.int64), torch.zeros(2, dtype=torch.int32),
                    torch.zeros(2, dtype=torch.float64))
