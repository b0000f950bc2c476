"""Python binding of the RSAI(tol) C ABI (``include/rsai.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``librsai.so``. PyTorch supplies device memory (its caching allocator is plugged
into the library) and streams. There is no CPU fallback: without the built library
or without a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RSAI_LIB") or os.path.join(_HERE, "librsai.so")

RSAI_OK = 0
_STATUS = {-1: "RSAI_E_ARG", -2: "RSAI_E_CSC", -3: "RSAI_E_SINGULAR", -4: "RSAI_E_NOMEM", -5: "RSAI_E_HIP",
           -6: "RSAI_E_CAP", -7: "RSAI_E_STATE"}
DROP = {"none": 0, "fixed": 1, "adaptive": 2}
SCHED = {"batched": 0, "plain": 1}


class RSAIError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("c", ctypes.c_int32), ("lmax", ctypes.c_int32), ("eps", ctypes.c_double),
                ("drop", ctypes.c_int32), ("tol", ctypes.c_double), ("sched", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("tier0", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("route", ctypes.c_int32),
                ("keep_factors", ctypes.c_int32), ("factor_budget_bytes", ctypes.c_int64),
                ("deterministic", ctypes.c_int32), ("tune_count", ctypes.c_int32),
                ("tune_table", ctypes.c_void_p), ("t0_hash", ctypes.c_int32), ("last_tier", ctypes.c_int32),
                ("col_len_max", ctypes.c_void_p), ("spill_capacity", ctypes.c_int64)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("len_lo", ctypes.c_double), ("len_hi", ctypes.c_double), ("eps_lo", ctypes.c_double),
                ("eps_hi", ctypes.c_double), ("maxlen_lo", ctypes.c_int64),
                ("maxlen_hi", ctypes.c_int64), ("n_lo", ctypes.c_int64), ("n_hi", ctypes.c_int64),
                ("tier0", ctypes.c_int32), ("refill", ctypes.c_int32), ("route", ctypes.c_int32),
                ("t0_hash", ctypes.c_int32), ("last_tier", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CSCView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("colptr", ctypes.c_void_p),
                ("rowidx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


_lib = None
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


_alloc_error = []


def _torch_alloc(size, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(size), torch.cuda.current_device(), stream or 0)
    except Exception as e:  # -> NULL; the library reports RSAI_E_NOMEM
        _alloc_error.append(repr(e))
        return None


def _torch_free(ptr, stream, ctx):
    if ptr:
        torch.cuda.caching_allocator_delete(ptr)


_alloc_cb = _ALLOC_T(_torch_alloc)
_free_cb = _FREE_T(_torch_free)


def load():
    """Load ``librsai.so`` and route its device allocations through PyTorch."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sigs = {
        "rsai_params_default": [P],
        "rsai_set_allocator": [P, P, P],
        "rsai_build": [P, P, P, P],
        "rsai_build_batched": [I32, P, P, P, P],
        "rsai_plan_count": [P, P],
        "rsai_plan_nnz": [P, I32, P],
        "rsai_export_M": [P, I32, P, P, P, P],
        "rsai_export_stats": [P, I32, P, P, P, P, P, P, P],
        "rsai_apply": [P, I32, P, P, P],
        "rsai_backward": [P, I32, P, D, P, P],
        "rsai_bicgstab": [P, I32, P, P, D, I32, I32, I32, P, P, P],
        "rsai_bicgstab_left": [P, P, I32, P, P, D, I32, I32, P, P, P],
        "rsai_transpose": [P, P, P, P, P],
        "rsai_spmv": [P, P, P, I32, P],
        "rsai_spmv_noalloc": [P, P, P, I32, P],
        "rsai_transversal": [P, P, P, P],
        "rsai_permute_rows": [P, P, P, P, P, P],
        "rsai_spmv_vjp": [P, P, P, P, P],
        "rsai_plan_timing": [P, P, I32],
        "rsai_peak_fp64": [I64, P, P],
        "rsai_tier_info": [I32, P, P, P],
        "rsai_rebuild": [P, I32, P],
        "rsai_autotune": [P, P, I32, P, P, I32, P, P],
        "rsai_plan_schedule": [P, P, P, P, P, P],
        "rsai_destroy": [P],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.rsai_last_error.argtypes = []
    lib.rsai_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code):
    if code != RSAI_OK:
        msg = load().rsai_last_error().decode()
        if code == -4 and _alloc_error:
            msg += f" (allocator: {_alloc_error[-1]})"
        raise RSAIError(code, msg)


def _use_torch_allocator():
    lib = load()
    _check(lib.rsai_set_allocator(ctypes.cast(_alloc_cb, ctypes.c_void_p), ctypes.cast(_free_cb, ctypes.c_void_p),
                                  None))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t.contiguous()


class Matrix:
    """A CSC matrix resident on the GPU (int64 colptr, int32 rowidx, float64 val)."""

    def __init__(self, colptr, rowidx, val):
        self.colptr = _dev(colptr, torch.int64, "colptr")
        self.rowidx = _dev(rowidx, torch.int32, "rowidx")
        self.val = _dev(val, torch.float64, "val")
        self.n = self.colptr.numel() - 1
        self.nnz = self.rowidx.numel()
        self._max_col_len = None

    @classmethod
    def from_host(cls, A, device="cuda"):
        M = cls(torch.as_tensor(A.colptr, dtype=torch.int64).to(device),
                torch.as_tensor(A.rowidx, dtype=torch.int32).to(device),
                torch.as_tensor(A.val, dtype=torch.float64).to(device))
        cp = A.colptr
        M._max_col_len = int((cp[1:] - cp[:-1]).max()) if len(cp) > 1 else 0
        return M

    @property
    def max_col_len(self):
        """Longest column (computed once; one device synchronisation if not known)."""
        if self._max_col_len is None:
            self._max_col_len = int((self.colptr[1:] - self.colptr[:-1]).max().item())
        return self._max_col_len

    def view(self, val=None):
        v = self.val if val is None else val
        return CSCView(self.n, self.nnz, self.colptr.data_ptr(), self.rowidx.data_ptr(), v.data_ptr())

    def transpose(self):
        """A^T on the same device (rsai_transpose)."""
        cp = torch.empty(self.n + 1, dtype=torch.int64, device=self.colptr.device)
        ri = torch.empty(self.nnz, dtype=torch.int32, device=self.colptr.device)
        va = torch.empty(self.nnz, dtype=torch.float64, device=self.colptr.device)
        v = self.view()
        _check(load().rsai_transpose(ctypes.byref(v), cp.data_ptr(), ri.data_ptr(), va.data_ptr(), _stream()))
        return Matrix(cp, ri, va)


def transversal(A: Matrix):
    """Maximum transversal of A's pattern (rsai_transversal): returns (p, size), p an
    int32 GPU tensor with p[k] the row matched to column k (-1 if none)."""
    _use_torch_allocator()
    p = torch.empty(A.n, dtype=torch.int32, device=A.colptr.device)
    size = ctypes.c_int64(0)
    v = A.view()
    _check(load().rsai_transversal(ctypes.byref(v), p.data_ptr(), ctypes.byref(size), _stream()))
    return p, size.value


def permute_rows(A: Matrix, p) -> Matrix:
    """P A: row p[k] of A becomes row k (rsai_permute_rows)."""
    _use_torch_allocator()
    p = _dev(p, torch.int32, "p")
    dev = A.colptr.device
    cp = torch.empty(A.n + 1, dtype=torch.int64, device=dev)
    ri = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    va = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev)
    v = A.view()
    _check(load().rsai_permute_rows(ctypes.byref(v), p.data_ptr(), cp.data_ptr(), ri.data_ptr(), va.data_ptr(),
                                    _stream()))
    return Matrix(cp, ri[:A.nnz], va[:A.nnz])


_params_memo = {}


def params(c=3, lmax=10, eps=0.4, drop="fixed", tol=1e-3, sched="batched", validate=True, tier0=-1,
           timing=False, refill=-1, route=-1, keep_factors=False, factor_budget_bytes=0, deterministic=False,
           t0_hash=-1, last_tier=-1, spill_capacity=0):
    # a fresh copy of the struct made earlier for the same arguments (the build is often
    # called in a loop with one parameter set)
    key = (c, lmax, eps, drop, tol, sched, validate, tier0, timing, refill, route, keep_factors,
           factor_budget_bytes, deterministic, t0_hash, last_tier, spill_capacity)
    try:
        made = _params_memo.get(key)
    except TypeError:  # unhashable argument: no memo
        key, made = None, None
    if made is not None:
        return Params.from_buffer_copy(made)
    p = _make_params(c, lmax, eps, drop, tol, sched, validate, tier0, timing, refill, route, keep_factors,
                     factor_budget_bytes, deterministic, t0_hash, last_tier, spill_capacity)
    if key is not None:
        if len(_params_memo) >= 256:
            _params_memo.clear()
        _params_memo[key] = bytes(p)
    return p


def _make_params(c, lmax, eps, drop, tol, sched, validate, tier0, timing, refill, route, keep_factors,
                 factor_budget_bytes, deterministic, t0_hash, last_tier, spill_capacity):
    p = Params()
    _check(load().rsai_params_default(ctypes.byref(p)))
    p.c, p.lmax, p.eps, p.tol = int(c), int(lmax), float(eps), float(tol)
    p.drop = DROP[drop] if isinstance(drop, str) else int(drop)
    p.sched = SCHED[sched] if isinstance(sched, str) else int(sched)
    p.validate = int(validate) if not isinstance(validate, bool) else (1 if validate else 0)
    p.tier0 = int(tier0)
    p.timing = 1 if timing else 0
    p.refill = int(refill)
    p.route = int(route)
    p.keep_factors = 1 if keep_factors else 0
    p.factor_budget_bytes = int(factor_budget_bytes)
    p.deterministic = 1 if deterministic else 0
    p.t0_hash = int(t0_hash)
    p.last_tier = int(last_tier)
    p.spill_capacity = int(spill_capacity)
    return p


class Plan:
    """Result of rsai_build / rsai_build_batched (owns the library plan)."""

    def __init__(self, handle, mats, prm, stream):
        self._h = handle
        self.mats = mats
        self.params = prm
        self.stream = stream

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rsai_destroy(h)
        self._h = None

    def _hv(self):
        if not self._h:
            raise RSAIError(-7, "plan is closed")
        return self._h

    def nnz(self, mat=0):
        out = ctypes.c_int64(0)
        _check(load().rsai_plan_nnz(self._hv(), mat, ctypes.byref(out)))
        return out.value

    def export(self, mat=0):
        """M of matrix mat as CSC tensors (colptr int64, rowidx int32, val float64)."""
        n = self.mats[mat].n
        nz = self.nnz(mat)
        dev = self.mats[mat].colptr.device
        cp = torch.empty(n + 1, dtype=torch.int64, device=dev)
        ri = torch.empty(max(nz, 1), dtype=torch.int32, device=dev)
        va = torch.empty(max(nz, 1), dtype=torch.float64, device=dev)
        _check(load().rsai_export_M(self._hv(), mat, cp.data_ptr(), ri.data_ptr(), va.data_ptr(), _stream()))
        return cp, ri[:nz], va[:nz]

    _STATS = {"loops": torch.int32, "resnorm": torch.float64, "nI": torch.int32, "nJ": torch.int32,
              "flops": torch.float64, "status": torch.int32}

    def stats(self, mat=0, fields=None):
        """Per-column statistics of matrix mat (rsai_export_stats); fields names the ones
        to export (default all of loops, resnorm, nI, nJ, flops, status)."""
        n = self.mats[mat].n
        dev = self.mats[mat].colptr.device
        names = tuple(self._STATS) if fields is None else tuple(fields)
        unknown = [f for f in names if f not in self._STATS]
        if unknown:
            raise ValueError(f"unknown statistics {unknown}")
        t = {k: torch.empty(n, dtype=self._STATS[k], device=dev) for k in names}
        ptr = {k: (t[k].data_ptr() if k in t else None) for k in self._STATS}
        _check(load().rsai_export_stats(self._hv(), mat, ptr["loops"], ptr["resnorm"], ptr["nI"], ptr["nJ"],
                                        ptr["flops"], ptr["status"], _stream()))
        return t

    def apply(self, x, mat=0):
        x = _dev(x, torch.float64, "x")
        y = torch.empty_like(x)
        _check(load().rsai_apply(self._hv(), mat, x.data_ptr(), y.data_ptr(), _stream()))
        return y

    def bicgstab(self, b, tol=1e-8, maxit=1000, precond=True, graph=True, mat=0):
        """Solve A x = b by BiCGStab right-preconditioned with M (rsai_bicgstab).
        Returns (x, iterations, relative residual); iterations is -1 on a breakdown
        and maxit + 1 without convergence."""
        b = _dev(b, torch.float64, "b")
        x = torch.empty_like(b)
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        _check(load().rsai_bicgstab(self._hv(), mat, b.data_ptr(), x.data_ptr(), float(tol), int(maxit),
                                    1 if precond else 0, 1 if graph else 0, ctypes.byref(it),
                                    ctypes.byref(rel), _stream()))
        return x, it.value, rel.value

    def backward(self, dM_val, w_frob, dA_val, mat=0):
        """dA_val += adjoint(dM_val) + w_frob * d(sum_k ||A m_k - e_k||^2)/dA (in place)."""
        dA_val = _dev(dA_val, torch.float64, "dA_val")
        ptr = None
        if dM_val is not None:
            dM_val = _dev(dM_val, torch.float64, "dM_val")
            ptr = dM_val.data_ptr()
        _check(load().rsai_backward(self._hv(), mat, ptr, float(w_frob), dA_val.data_ptr(), _stream()))
        return dA_val

    def rebuild(self, graph=True, stream=None):
        """Run the build again with the values the plan's matrices hold now
        (rsai_rebuild; graph=True replays a captured HIP graph)."""
        _check(load().rsai_rebuild(self._hv(), 1 if graph else 0, _stream(stream)))

    def schedule(self):
        """The schedule the build used (rsai_plan_schedule)."""
        v = [ctypes.c_int32() for _ in range(5)]
        _check(load().rsai_plan_schedule(self._hv(), *[ctypes.byref(x) for x in v]))
        return dict(zip(("tier0", "refill", "route", "t0_hash", "last_tier"), (x.value for x in v)))

    def timing(self):
        ms = (ctypes.c_double * 6)()
        _check(load().rsai_plan_timing(self._hv(), ms, 6))
        return {"prep": ms[0], "tier0": ms[1], "tiers": ms[2], "assemble": ms[3], "build": ms[4], "backward": ms[5]}


def build(A: Matrix, stream=None, **kw) -> Plan:
    """Build the sparse approximate inverse M of one matrix (rsai_build)."""
    return build_batched([A], stream=stream, **kw)


_tune_memo = [None, None, 0]  # entries list converted last, its array, count


def tune_entries(table=None):
    """The tuning table (tune.load_table entries, or the given list of dicts) as the C
    ABI's rsai_tune_entry array; fields an entry lacks are -1 (not applied)."""
    from . import tune
    rows = tune.load_table() if table is None else table
    if table is None and _tune_memo[0] is rows:
        return _tune_memo[1], _tune_memo[2]
    arr = (TuneEntry * max(len(rows), 1))()
    for i, e in enumerate(rows):
        arr[i] = TuneEntry(float(e["len_lo"]), float(e["len_hi"]), float(e.get("eps_lo", 0.0)),
                           float(e.get("eps_hi", float("inf"))), int(e["maxlen_lo"]), int(e["maxlen_hi"]),
                           int(e["n_lo"]), int(e["n_hi"]), int(e.get("tier0", -1)), int(e.get("refill", -1)),
                           int(e.get("route", -1)), int(e.get("t0_hash", -1)), int(e.get("last_tier", -1)), 0)
    if table is None:
        _tune_memo[:] = [rows, arr, len(rows)]
    return arr, len(rows)


def build_batched(mats, stream=None, tune_table=None, **kw) -> Plan:
    """Build M for several matrices in one pass (rsai_build_batched). The tuning table
    (tuning.json, or tune_table: a list of entries; [] for none) goes to the library
    through rsai_params, which applies it to the schedule fields left at -1."""
    lib = load()
    _use_torch_allocator()
    prm = params(**kw)
    entries, count = tune_entries(tune_table)
    if count:
        prm.tune_table = ctypes.cast(entries, ctypes.c_void_p)
        prm.tune_count = count
    # the longest column of each matrix, when the host knows it (saves the library a
    # device read and a synchronisation)
    lens = None
    if count and all(m._max_col_len is not None for m in mats):
        lens = (ctypes.c_int64 * len(mats))(*[int(m._max_col_len) for m in mats])
        prm.col_len_max = ctypes.cast(lens, ctypes.c_void_p)
    views = (CSCView * len(mats))(*[m.view() for m in mats])
    h = ctypes.c_void_p()
    st = _stream(stream)
    _check(lib.rsai_build_batched(len(mats), views, ctypes.byref(prm), st, ctypes.byref(h)))
    prm.tune_table = None  # the table and the lengths are read during the call only
    prm.tune_count = 0
    prm.col_len_max = None
    return Plan(h, list(mats), prm, st)


def bicgstab_left(A: Matrix, plan_t: "Plan", b, tol=1e-8, maxit=1000, graph=True, mat=0):
    """Solve M A x = b's left-preconditioned form M A x = M b by BiCGStab, with M the
    transpose of the RSAI factor of A^T (plan_t built on A.transpose()); the test is
    ||b - A x|| / ||b|| < tol (rsai_bicgstab_left). Returns (x, iterations, relres)."""
    b = _dev(b, torch.float64, "b")
    x = torch.empty_like(b)
    it = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    v = A.view()
    _check(load().rsai_bicgstab_left(ctypes.byref(v), plan_t._hv(), mat, b.data_ptr(), x.data_ptr(), float(tol),
                                     int(maxit), 1 if graph else 0, ctypes.byref(it), ctypes.byref(rel), _stream()))
    return x, it.value, rel.value


def spmv(A: Matrix, x, transpose=False, val=None):
    """y = A x or A^T x (rsai_spmv)."""
    x = _dev(x, torch.float64, "x")
    y = torch.empty(A.n, dtype=torch.float64, device=x.device)
    v = A.view(val)
    _check(load().rsai_spmv(ctypes.byref(v), x.data_ptr(), y.data_ptr(), 1 if transpose else 0, _stream()))
    return y


def spmv_noalloc(A: Matrix, x, y, transpose=False, val=None):
    """y = A x or A^T x into the caller's y without any allocation (rsai_spmv_noalloc)."""
    x = _dev(x, torch.float64, "x")
    if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == torch.float64 and y.is_contiguous()
            and y.numel() == A.n):
        raise ValueError("y must be a contiguous float64 GPU tensor of n entries")
    v = A.view(val)
    _check(load().rsai_spmv_noalloc(ctypes.byref(v), x.data_ptr(), y.data_ptr(), 1 if transpose else 0, _stream()))
    return y


def spmv_vjp(A: Matrix, dy, x, dval, val=None):
    """dval[e] += dy[i] * x[j] for each stored entry (i, j) of A (rsai_spmv_vjp)."""
    dy = _dev(dy, torch.float64, "dy")
    x = _dev(x, torch.float64, "x")
    dval = _dev(dval, torch.float64, "dval")
    v = A.view(val)
    _check(load().rsai_spmv_vjp(ctypes.byref(v), dy.data_ptr(), x.data_ptr(), dval.data_ptr(), _stream()))
    return dval


def peak_fp64(iters=1 << 16) -> float:
    """Measured FP64 vector FMA rate of the current device in TFLOP/s (rsai_peak_fp64)."""
    _use_torch_allocator()
    out = ctypes.c_double()
    _check(load().rsai_peak_fp64(int(iters), ctypes.byref(out), _stream()))
    return out.value


def tier_info(t):
    g, mr, mc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().rsai_tier_info(t, ctypes.byref(g), ctypes.byref(mr), ctypes.byref(mc)))
    return g.value, mr.value, mc.value
