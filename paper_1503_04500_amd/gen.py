"""Seeded synthetic sparse matrices in CSC form.

This module only builds inputs. It holds none of the sparse-approximate-inverse
arithmetic and is shared by the tests, the CPU oracle's callers and the benchmark.

The matrices stand in for the paper's test matrices (Section 5, Table 1), which are
collection matrices not available here:

* ``cd2d`` / ``cd3d``: h^2-scaled 5-/7-point upwind convection-diffusion operators on
  the unit square/cube with Dirichlet boundaries, lexicographic numbering
  k = ix + N*iy (+ N^2*iz). They are regular sparse (a few nonzeros per column, like
  the reservoir-simulation matrices of Table 1).
* ``powerlaw``: a random nonsymmetric matrix whose column lengths follow a power
  law, i.e. a column-irregular matrix in the sense of Section 1 (some columns have
  far more than 10 p nonzeros, p the mean per column).
* ``batch64``: 64 matrices of the three kinds with log-uniform sizes.

CSC layout: int64 colptr[n+1], int32 rowidx[nnz] (ascending and unique inside each
column), float64 val[nnz].
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

__all__ = ["CSC", "cd2d", "cd3d", "powerlaw", "batch64_specs", "make", "c1", "c2",
           "c3", "c4", "tridiag", "diagonal", "POWERLAW_ALPHA"]

# Exponent of P(L) ~ L^-alpha on {2..200} whose mean column length is 7.00.
POWERLAW_ALPHA = 2.0603


@dataclasses.dataclass
class CSC:
    n: int
    colptr: np.ndarray  # int64 [n+1]
    rowidx: np.ndarray  # int32 [nnz]
    val: np.ndarray     # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (np.ascontiguousarray(self.colptr, np.int64),
                  np.ascontiguousarray(self.rowidx, np.int32),
                  np.ascontiguousarray(self.val, np.float64)):
            h.update(a.tobytes())
        return h.hexdigest()

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        for j in range(self.n):
            s, e = self.colptr[j], self.colptr[j + 1]
            d[self.rowidx[s:e], j] = self.val[s:e]
        return d

    def col_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.colptr))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        y = np.zeros(self.n)
        np.add.at(y, self.rowidx, self.val * x[self.col_of_entry()])
        return y

    def with_values(self, val: np.ndarray) -> "CSC":
        return CSC(self.n, self.colptr, self.rowidx, np.ascontiguousarray(val, np.float64), self.name)


def from_coo(n: int, rows, cols, vals, name: str = "") -> CSC:
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    vals = np.asarray(vals, np.float64)
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate COO entries")
    colptr = np.zeros(n + 1, np.int64)
    np.add.at(colptr, cols + 1, 1)
    np.cumsum(colptr, out=colptr)
    return CSC(n, colptr, rows.astype(np.int32), vals, name)


def from_dense(d: np.ndarray, name: str = "") -> CSC:
    r, c = np.nonzero(d.T)  # column-major walk
    return from_coo(d.shape[0], c, r, d[c, r], name)


def _stencil(shape, b, h):
    """Upwind h^2-scaled convection-diffusion stencil.

    ``b`` is (n, dim): the convection vector at each cell (the row's cell). Along
    each axis the neighbour on the upwind side (the side the flow comes from) gets
    -1 - |b_d| h, the other neighbour -1, and the diagonal 2*dim + sum_d |b_d| h.
    """
    dim = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for N in shape:
        coords.append(rem % N)
        rem //= N
    strides = [1]
    for N in shape[:-1]:
        strides.append(strides[-1] * N)
    rows, cols, vals = [idx], [idx], [2.0 * dim + np.abs(b).sum(axis=1) * h]
    for d in range(dim):
        bd = b[:, d]
        for sgn in (-1, +1):
            nb = coords[d] + sgn
            ok = (nb >= 0) & (nb < shape[d])
            # flow along +axis (bd > 0) comes from the minus side
            upwind = (bd > 0) if sgn < 0 else (bd < 0)
            v = -1.0 - np.where(upwind, np.abs(bd) * h, 0.0)
            rows.append(idx[ok])
            cols.append(idx[ok] + sgn * strides[d])
            vals.append(v[ok])
    return n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def cd2d(N: int, conv=None, seed: int | None = 0, lo: float = -50.0, hi: float = 50.0) -> CSC:
    """2D 5-point convection-diffusion on an N x N grid, h = 1/(N+1).

    ``conv=(bx, by)`` gives a constant convection; otherwise each cell draws
    (bx, by) uniform in [lo, hi]^2 from ``default_rng(seed)``.
    """
    h = 1.0 / (N + 1)
    n = N * N
    if conv is not None:
        b = np.tile(np.asarray(conv, np.float64), (n, 1))
    else:
        b = np.random.default_rng(seed).uniform(lo, hi, (n, 2))
    n, r, c, v = _stencil((N, N), b, h)
    return from_coo(n, r, c, v, f"cd2d_{N}")


def cd3d(N: int, conv=None, seed: int | None = 0, lo: float = -50.0, hi: float = 50.0) -> CSC:
    """3D 7-point convection-diffusion on an N^3 grid, h = 1/(N+1)."""
    h = 1.0 / (N + 1)
    n = N ** 3
    if conv is not None:
        b = np.tile(np.asarray(conv, np.float64), (n, 1))
    else:
        b = np.random.default_rng(seed).uniform(lo, hi, (n, 3))
    n, r, c, v = _stencil((N, N, N), b, h)
    return from_coo(n, r, c, v, f"cd3d_{N}")


def powerlaw(n: int, seed: int = 0, lmin: int = 2, lmax: int = 200,
             alpha: float = POWERLAW_ALPHA, diag_factor: float = 1.2) -> CSC:
    """Random nonsymmetric matrix with power-law column lengths.

    Column k has L_k entries, L_k iid with P(L) proportional to L^-alpha on
    {lmin..lmax} (L_k counts the diagonal). Its L_k - 1 off-diagonal rows are
    distinct and uniform over {0..n-1} minus {k}; their values are N(0,1). The
    diagonal is diag_factor times the column's off-diagonal absolute sum.
    """
    rng = np.random.default_rng(seed)
    Ls = np.arange(lmin, min(lmax, n) + 1)
    p = Ls.astype(np.float64) ** (-alpha)
    p /= p.sum()
    L = rng.choice(Ls, size=n, p=p).astype(np.int64)
    off = L - 1
    cols = np.repeat(np.arange(n, dtype=np.int64), off)
    rows = rng.integers(0, n - 1, size=cols.size)
    rows = rows + (rows >= cols)  # uniform over {0..n-1} minus {col}
    while True:
        order = np.lexsort((rows, cols))
        rows, cols = rows[order], cols[order]
        dup = np.zeros(rows.size, bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        nd = int(dup.sum())
        if nd == 0:
            break
        redraw = rng.integers(0, n - 1, size=nd)
        rows[dup] = redraw + (redraw >= cols[dup])
    vals = rng.standard_normal(rows.size)
    absum = np.zeros(n)
    np.add.at(absum, cols, np.abs(vals))
    diag = diag_factor * absum
    allr = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    allc = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    allv = np.concatenate([vals, diag])
    return from_coo(n, allr, allc, allv, f"powerlaw_{n}")


def dense_rows(N: int, nrows: int, rowlen: int, scale: float = 1.0, seed: int = 0) -> CSC:
    """2D convection-diffusion matrix (cd2d(N, seed)) with nrows relatively dense rows.

    Each chosen row (distinct, uniform) gets rowlen - 1 extra off-diagonal entries in
    distinct uniform columns not already in the row, values scale * U(-1, 1). Such
    rows pull their whole pattern into J_k when they are selected as dominant, which
    is the regime where the LS problems grow large (Section 4).
    """
    base = cd2d(N, seed=seed)
    n = base.n
    rng = np.random.default_rng(seed + 7919)
    rows = [base.rowidx.astype(np.int64)]
    cols = [base.col_of_entry().astype(np.int64)]
    vals = [base.val]
    have = set(zip(rows[0].tolist(), cols[0].tolist()))
    for i in rng.choice(n, size=nrows, replace=False):
        picked = []
        while len(picked) < rowlen - 1:
            j = int(rng.integers(0, n))
            if j != i and (int(i), j) not in have:
                have.add((int(i), j))
                picked.append(j)
        rows.append(np.full(len(picked), i, np.int64))
        cols.append(np.asarray(picked, np.int64))
        vals.append(scale * rng.uniform(-1.0, 1.0, len(picked)))
    return from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                    f"dense_rows_{N}_{nrows}_{rowlen}")


def tridiag(n: int, lower: float = -1.0, diag: float = 2.0, upper: float = -1.0) -> CSC:
    d = np.diag(np.full(n, diag)) + np.diag(np.full(n - 1, lower), -1) + np.diag(np.full(n - 1, upper), 1)
    return from_dense(d, f"tridiag_{n}")


def diagonal(d) -> CSC:
    d = np.asarray(d, np.float64)
    n = d.size
    return from_coo(n, np.arange(n), np.arange(n), d, f"diag_{n}")


def batch64_specs(count: int = 64, nmin: int = 4096, nmax: int = 262144):
    """Specs of the multi-matrix batch: kind cycles cd2d, cd3d, powerlaw; n log-uniform."""
    kinds = ("cd2d", "cd3d", "powerlaw")
    specs = []
    for i in range(count):
        rng = np.random.default_rng(1000 + i)
        ni = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kind = kinds[i % 3]
        if kind == "cd2d":
            N = max(2, int(round(ni ** 0.5)))
            specs.append(("cd2d", N, 3000 + i))
        elif kind == "cd3d":
            N = max(2, int(round(ni ** (1.0 / 3.0))))
            specs.append(("cd3d", N, 3000 + i))
        else:
            specs.append(("powerlaw", ni, 3000 + i))
    return specs


def make(spec) -> CSC:
    kind, size, seed = spec
    if kind == "cd2d":
        return cd2d(size, seed=seed)
    if kind == "cd3d":
        return cd3d(size, seed=seed)
    if kind == "powerlaw":
        return powerlaw(size, seed=seed)
    raise ValueError(kind)


def c1() -> CSC:
    """32x32 grid, constant convection (10, 5): n = 1024, nnz = 4992."""
    return cd2d(32, conv=(10.0, 5.0))


def c2(N: int = 512) -> CSC:
    """512x512 grid, per-cell convection U[-50,50]^2 (seed 0): n = 262144."""
    return cd2d(N, seed=0)


def c3(n: int = 1_000_000) -> CSC:
    """Power-law columns (min 2, mean 7, max 200), n = 10^6, seed 0."""
    return powerlaw(n, seed=0)


def c4(N: int = 64) -> CSC:
    """64^3 grid, per-cell convection U[-50,50]^3 (seed 0): n = 262144."""
    return cd3d(N, seed=0)
