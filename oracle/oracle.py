"""ctypes wrapper of the plain C oracle (``rsai_oracle.c``) -- test infrastructure only.

Inputs are CSC arrays (int64 colptr, int32 rowidx, float64 val); see the C file for
the method and the conventions taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

DROP_NONE, DROP_FIXED, DROP_ADAPTIVE = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsai_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double


def build_lib(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_lib(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.oracle_rsai.restype = _P
    lib.oracle_rsai.argtypes = [_I64, _P, _P, _P, _I32, _I32, _D, _I32, _D, _I32, _P, _I64, _I32]
    lib.oracle_nnz.restype = _I64
    lib.oracle_nnz.argtypes = [_P]
    lib.oracle_seconds.restype = _D
    lib.oracle_seconds.argtypes = [_P]
    lib.oracle_threads.restype = _I32
    lib.oracle_threads.argtypes = [_P]
    lib.oracle_export.restype = None
    lib.oracle_export.argtypes = [_P] * 16
    lib.oracle_export_peaks.restype = None
    lib.oracle_export_peaks.argtypes = [_P] * 3
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [_P]
    lib.oracle_fixed_pattern.restype = _I64
    lib.oracle_fixed_pattern.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _I32]
    lib.oracle_backward.restype = _I64
    lib.oracle_backward.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _P, _P]
    lib.oracle_bicgstab.restype = _I32
    lib.oracle_bicgstab.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _I32, _P, _P]
    lib.oracle_bicgstab_left.restype = _I32
    lib.oracle_bicgstab_left.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _I32, _P, _P]
    lib.oracle_transversal.restype = _I64
    lib.oracle_transversal.argtypes = [_I64, _P, _P, _P]
    lib.oracle_model_solve_flops.restype = _D
    lib.oracle_model_solve_flops.argtypes = [_I32, _I32, _I32, _I32]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csc(colptr, rowidx, val):
    return (np.ascontiguousarray(colptr, np.int64), np.ascontiguousarray(rowidx, np.int32),
            np.ascontiguousarray(val, np.float64))


def rsai(A, c: int = 3, lmax: int = 8, eps: float = 0.4, drop: int = DROP_FIXED, tol: float = 1e-3,
         threads: int = 0, cols=None, hist: bool = False) -> dict:
    """RSAI(tol) per Algorithm 1 with dropping. ``A`` has n, colptr, rowidx, val.

    Returns a dict with the CSC of M (columns = the processed columns, ascending) and
    per-column statistics: loops, resnorm (||A m_k - e_k||), nI, nJ, status,
    sel_margin / drop_margin (smallest decision gaps), flops (the oracle's own
    from-scratch count), mflops (the QR-update work model), nsolve (loop solves),
    ndrop (re-solves after a drop), nImax / nJmax (the largest |I_k|, |J_k| of any
    solve, i.e. before a drop shrinks J_k), and optionally hist (residual norm after
    each loop solve).
    """
    if not (1 <= c <= 64):
        raise ValueError("c must be in 1..64")
    lib = _load()
    cp, ri, va = _csc(A.colptr, A.rowidx, A.val)
    n = int(A.n)
    colsa = None if cols is None else np.ascontiguousarray(np.sort(np.asarray(cols, np.int64)))
    ncols = n if colsa is None else colsa.size
    h = lib.oracle_rsai(n, _ptr(cp), _ptr(ri), _ptr(va), c, lmax, eps, drop, tol, threads,
                        _ptr(colsa), ncols, 1 if hist else 0)
    if not h:
        raise MemoryError("oracle_rsai failed")
    try:
        nnz = lib.oracle_nnz(h)
        out = dict(
            colptr=np.zeros(ncols + 1, np.int64), rowidx=np.zeros(nnz, np.int32), val=np.zeros(nnz),
            loops=np.zeros(ncols, np.int32), resnorm=np.zeros(ncols), nI=np.zeros(ncols, np.int32),
            nJ=np.zeros(ncols, np.int32), status=np.zeros(ncols, np.int32), sel_margin=np.zeros(ncols),
            drop_margin=np.zeros(ncols), flops=np.zeros(ncols), nsolve=np.zeros(ncols, np.int32),
            ndrop=np.zeros(ncols, np.int32), mflops=np.zeros(ncols))
        hh = np.zeros(ncols * 2 * (lmax + 1)) if hist else None
        lib.oracle_export(h, *[_ptr(out[k]) for k in ("colptr", "rowidx", "val", "loops", "resnorm", "nI",
                                                      "nJ", "status", "sel_margin", "drop_margin", "flops",
                                                      "nsolve")], _ptr(hh), _ptr(out["ndrop"]),
                           _ptr(out["mflops"]))
        out["nImax"] = np.zeros(ncols, np.int32)
        out["nJmax"] = np.zeros(ncols, np.int32)
        lib.oracle_export_peaks(h, _ptr(out["nImax"]), _ptr(out["nJmax"]))
        if hist:
            out["hist"] = hh.reshape(ncols, 2 * (lmax + 1))
        out["seconds"] = lib.oracle_seconds(h)
        out["threads"] = lib.oracle_threads(h)
        out["cols"] = np.arange(n) if colsa is None else colsa
        out["n"] = n
        return out
    finally:
        lib.oracle_free(h)


def model_solve_flops(m0: int, m: int, qlo: int, qn: int) -> float:
    """The QR-update work model of one LS solve: a factor of qlo columns formed on m0
    rows is kept and the block grows to m rows and qn columns (qlo = 0: from scratch)."""
    return float(_load().oracle_model_solve_flops(int(m0), int(m), int(qlo), int(qn)))


def transversal(A):
    """Maximum transversal of the pattern of A by augmenting paths. Returns (size,
    match) with match[k] the row matched to column k (-1 if unmatched); size == n
    gives a row permutation p = match with A(p[k], k) != 0 for every k."""
    lib = _load()
    cp, ri, _ = _csc(A.colptr, A.rowidx, A.val)
    match = np.full(int(A.n), -1, np.int32)
    size = lib.oracle_transversal(int(A.n), _ptr(cp), _ptr(ri), _ptr(match))
    if size < 0:
        raise MemoryError("oracle_transversal failed")
    return int(size), match


def permute_rows(A, p):
    """The rows of A renumbered by the permutation p: row p[k] of A becomes row k
    (B(k, j) = A(p[k], j)). Returns B as CSC arrays (colptr, rowidx, val), rows
    ascending in every column."""
    p = np.asarray(p, np.int64)
    n = int(A.n)
    if p.shape != (n,) or not np.array_equal(np.sort(p), np.arange(n)):
        raise ValueError("p must be a permutation of 0..n-1")
    inv = np.empty(n, np.int64)
    inv[p] = np.arange(n)
    cp, ri, va = _csc(A.colptr, A.rowidx, A.val)
    rows = inv[ri]
    col = np.repeat(np.arange(n), np.diff(cp))
    order = np.lexsort((rows, col))
    return cp.copy(), rows[order].astype(np.int32), va[order].copy()


def fixed_pattern(A, Mcolptr, Mrowidx, threads: int = 0):
    """Solve (2.3) for every column on the given pattern. Returns (Mval, resnorm)."""
    lib = _load()
    cp, ri, va = _csc(A.colptr, A.rowidx, A.val)
    mcp = np.ascontiguousarray(Mcolptr, np.int64)
    mri = np.ascontiguousarray(Mrowidx, np.int32)
    mval = np.zeros(mri.size)
    rn = np.zeros(int(A.n))
    bad = lib.oracle_fixed_pattern(int(A.n), _ptr(cp), _ptr(ri), _ptr(va), _ptr(mcp), _ptr(mri), _ptr(mval),
                                   _ptr(rn), threads)
    if bad:
        raise ArithmeticError(f"{bad} singular columns")
    return mval, rn


def backward(A, Mcolptr, Mrowidx, Mval, gM=None, w_frob: float = 0.0, scale: bool = False):
    """Adjoint of the fixed-pattern LS map: returns dL/d(values of A) (length nnz(A));
    with scale=True also, per entry, the sum of the magnitudes of the terms added into
    it (the yardstick of a per-entry rounding tolerance)."""
    lib = _load()
    cp, ri, va = _csc(A.colptr, A.rowidx, A.val)
    mcp = np.ascontiguousarray(Mcolptr, np.int64)
    mri = np.ascontiguousarray(Mrowidx, np.int32)
    mv = np.ascontiguousarray(Mval, np.float64)
    g = None if gM is None else np.ascontiguousarray(gM, np.float64)
    dA = np.zeros(va.size)
    sc = np.zeros(va.size) if scale else None
    bad = lib.oracle_backward(int(A.n), _ptr(cp), _ptr(ri), _ptr(va), _ptr(mcp), _ptr(mri), _ptr(mv), _ptr(g),
                              float(w_frob), _ptr(dA), _ptr(sc))
    if bad:
        raise ArithmeticError(f"{bad} singular columns")
    return (dA, sc) if scale else dA


def bicgstab(A, b, M=None, tol: float = 1e-8, maxit: int = 1000, left: bool = False):
    """BiCGStab preconditioned with M: on A M y = b (right, x = M y) or, with
    left=True, on M A x = M b. Returns (iterations, relres, x); the test is the true
    relative residual ||b - A x|| / ||b|| < tol after each half and full step.

    iterations = maxit + 1 means no convergence; -1 means breakdown.
    ``M`` is None or a (colptr, rowidx, val) tuple (required for left=True).
    """
    lib = _load()
    cp, ri, va = _csc(A.colptr, A.rowidx, A.val)
    bb = np.ascontiguousarray(b, np.float64)
    x = np.zeros(int(A.n))
    rel = ctypes.c_double(0.0)
    if M is None:
        mcp = mri = mv = None
    else:
        mcp, mri, mv = _csc(*M)
    if left and M is None:
        raise ValueError("left preconditioning needs M")
    fn = lib.oracle_bicgstab_left if left else lib.oracle_bicgstab
    it = fn(int(A.n), _ptr(cp), _ptr(ri), _ptr(va), _ptr(mcp), _ptr(mri), _ptr(mv), _ptr(bb),
            float(tol), int(maxit), _ptr(x), ctypes.byref(rel))
    return int(it), float(rel.value), x
