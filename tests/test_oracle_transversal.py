"""Pins of the oracle's maximum transversal (the row permutation to a zero-free
diagonal that Section 5 applies to its zero-diagonal matrices): brute force over
all permutations on tiny patterns, validity, structurally singular patterns with
a known structural rank (Hall's condition fails), and the permuted matrix."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen


def _valid(A, size, match):
    """match[k] is a stored row of column k or -1, rows distinct, size = #matched."""
    used = match[match >= 0]
    assert used.size == size and np.unique(used).size == size
    for k in np.nonzero(match >= 0)[0]:
        rows = A.rowidx[A.colptr[k]:A.colptr[k + 1]]
        assert match[k] in rows


def _brute_rank(d):
    """Largest number of nonzeros on the diagonal of any row permutation."""
    n = d.shape[0]
    nz = d != 0
    return max(sum(nz[s[k], k] for k in range(n)) for s in itertools.permutations(range(n)))


@pytest.mark.parametrize("seed", range(40))
def test_tiny_patterns_match_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 8))
    dens = rng.uniform(0.1, 0.6)
    d = np.where(rng.random((n, n)) < dens, rng.standard_normal((n, n)), 0.0)
    for k in range(n):  # every column keeps at least one entry (the CSC contract)
        if not d[:, k].any():
            d[rng.integers(n), k] = 1.0
    A = gen.from_dense(d)
    size, match = oracle.transversal(A)
    _valid(A, size, match)
    assert size == _brute_rank(d)


def test_structurally_singular_ranks():
    # two columns whose only entries share one row: rank n - 1 (Hall fails on them)
    n = 6
    d = np.eye(n) + np.diag((np.arange(n - 1) >= 2).astype(float), 1)
    d[:, 1] = 0.0
    d[0, 1] = 1.0   # columns 0 and 1 hold row 0 only
    A = gen.from_dense(d)
    size, match = oracle.transversal(A)
    _valid(A, size, match)
    assert size == n - 1
    # k columns living in k - 1 rows: rank n - 1
    d = np.eye(8)
    d[:, 5] = 0.0
    d[[3, 4], 5] = 1.0
    d[:, 3] = 0.0
    d[[3, 4], 3] = 1.0   # columns 3, 4, 5 only touch rows 3 and 4
    A = gen.from_dense(d)
    size, match = oracle.transversal(A)
    _valid(A, size, match)
    assert size == 7


def test_permutation_matrix_and_zero_diagonal_grid():
    n = 300
    pi = np.random.default_rng(1).permutation(n)
    P = gen.from_coo(n, pi, np.arange(n), np.ones(n))
    size, match = oracle.transversal(P)
    assert size == n and np.array_equal(match, pi)   # the only transversal
    A = gen.cd2d(24, seed=2)
    perm = np.random.default_rng(5).permutation(A.n)
    inv = np.empty(A.n, np.int64)
    inv[perm] = np.arange(A.n)
    B = gen.from_coo(A.n, inv[A.rowidx], A.col_of_entry(), A.val)
    assert (B.to_dense().diagonal() == 0).sum() == 567
    size, match = oracle.transversal(B)
    _valid(B, size, match)
    assert size == B.n
    cp, ri, va = oracle.permute_rows(B, match)
    C = gen.CSC(B.n, cp, ri, va)
    dC, dB = C.to_dense(), B.to_dense()
    assert np.all(dC.diagonal() != 0)
    assert np.array_equal(dC, dB[match, :])    # row k of C is row match[k] of B
    for k in range(C.n):
        assert np.all(np.diff(ri[cp[k]:cp[k + 1]]) > 0)


def test_permute_rows_rejects_non_permutations():
    A = gen.c1()
    with pytest.raises(ValueError):
        oracle.permute_rows(A, np.zeros(A.n, np.int64))
