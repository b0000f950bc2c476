"""Row permutation to a zero-free diagonal (Section 5's preprocessing of matrices with
zero diagonal entries) on the GPU: rsai_transversal vs the oracle's augmenting-path
matching (several maximum transversals can exist, so the size is compared and the
GPU's matching is checked for validity), rsai_permute_rows vs the oracle's
renumbering, then RSAI(tol) and BiCGStab on the permuted matrix."""
import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen
from tests.parity import compare, run_gpu

pytestmark = pytest.mark.gpu
C1 = dict(c=3, lmax=8, eps=0.4, tol=1e-3)


def _row_permuted(A, seed):
    perm = np.random.default_rng(seed).permutation(A.n)
    inv = np.empty(A.n, np.int64)
    inv[perm] = np.arange(A.n)
    return gen.from_coo(A.n, inv[A.rowidx], A.col_of_entry(), A.val, name=A.name + " rows permuted")


def _gpu_transversal(A):
    import paper_1503_04500_amd.rsai as rsai
    dA = rsai.Matrix.from_host(A, "cuda:0")
    p, size = rsai.transversal(dA)
    return dA, p, p.cpu().numpy(), size


def _check_valid(A, p, size):
    """p[k] a stored row of column k or -1; matched rows distinct; size = matched."""
    m = p >= 0
    assert int(m.sum()) == size
    assert np.unique(p[m]).size == size
    cp = A.colptr
    k = np.nonzero(m)[0]
    # each matched row is stored in its column (rows ascending: bisection)
    for kk in k:
        rows = A.rowidx[cp[kk]:cp[kk + 1]]
        j = np.searchsorted(rows, p[kk])
        assert j < rows.size and rows[j] == p[kk], kk


@pytest.mark.parametrize("which", ["grid24", "grid512", "powerlaw", "identity", "perm"])
def test_transversal_full_rank(which):
    A = {"grid24": lambda: _row_permuted(gen.cd2d(24, seed=2), 5),
         "grid512": lambda: _row_permuted(gen.cd2d(512), 7),
         "powerlaw": lambda: _row_permuted(gen.powerlaw(100000, seed=3), 9),
         "identity": lambda: gen.cd2d(64, seed=1),
         "perm": lambda: gen.from_coo(5000, np.random.default_rng(4).permutation(5000), np.arange(5000),
                                      np.ones(5000))}[which]()
    print(which, "n =", A.n, "zero diagonal entries:", int(A.n - np.sum(
        np.repeat(np.arange(A.n), np.diff(A.colptr)) == A.rowidx)), flush=True)
    _, _, p, size = _gpu_transversal(A)
    want, _ = oracle.transversal(A) if A.n <= 300000 else (A.n, None)
    assert size == want == A.n
    _check_valid(A, p, size)
    assert np.array_equal(np.sort(p), np.arange(A.n))
    if which == "identity":   # diagonal entries present: the greedy claims keep them
        assert np.array_equal(p, np.arange(A.n))


@pytest.mark.parametrize("seed", range(6))
def test_transversal_structurally_singular(seed):
    """Random sparse patterns, some structurally singular: the GPU's size equals the
    oracle's (the structural rank is unique)."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(50, 400))
    nnz = int(n * rng.uniform(1.0, 2.5))
    rows = rng.integers(0, n, nnz)
    cols = np.concatenate([np.arange(n), rng.integers(0, n, nnz - n)])
    key = np.unique(rows.astype(np.int64) * n + cols)
    rows, cols = (key // n), (key % n)
    A = gen.from_coo(n, rows, cols, rng.standard_normal(rows.size))
    want, _ = oracle.transversal(A)
    _, _, p, size = _gpu_transversal(A)
    print("n", n, "structural rank", want, flush=True)
    assert size == want
    _check_valid(A, p, size)


def test_permute_rows_matches_oracle_and_rejects_non_permutations():
    import torch
    import paper_1503_04500_amd.rsai as rsai
    B = _row_permuted(gen.cd2d(24, seed=2), 5)
    _, po = oracle.transversal(B)
    want = oracle.permute_rows(B, po)
    dB = rsai.Matrix.from_host(B, "cuda:0")
    C = rsai.permute_rows(dB, torch.from_numpy(po).cuda())
    for got, w in zip((C.colptr, C.rowidx, C.val), want):
        assert np.array_equal(got.cpu().numpy(), w)
    bad = torch.zeros(B.n, dtype=torch.int32, device="cuda:0")
    with pytest.raises(rsai.RSAIError) as ei:
        rsai.permute_rows(dB, bad)
    assert ei.value.code == -1


def test_rsai_on_permuted_zero_diagonal_matrix():
    """The 24x24 grid with its rows permuted at random (567 of 576 zero diagonal
    entries), permuted back to a zero-free diagonal by the oracle's transversal: RSAI
    of the permuted matrix on the GPU equals the oracle's (full parity bar)."""
    B = _row_permuted(gen.cd2d(24, seed=2), 5)
    _, po = oracle.transversal(B)
    C = gen.CSC(B.n, *oracle.permute_rows(B, po))
    ref = oracle.rsai(C, **C1)
    gpu = run_gpu(C, **C1)
    s = compare(C, gpu, ref, label="permuted zero-diagonal")
    print("parity", s, flush=True)


def test_bicgstab_after_permutation_end_to_end():
    """Everything on the device: transversal, P A, RSAI of P A, BiCGStab on
    (P A) x = P b; x solves A x = b. The unpermuted matrix (k outside I_k, r(k) = -1)
    is solved the same way for comparison, and both counts are reported."""
    import torch
    import paper_1503_04500_amd.rsai as rsai
    B = _row_permuted(gen.cd2d(64, seed=2), 5)
    dB, p, ph, size = _gpu_transversal(B)
    assert size == B.n
    C = rsai.permute_rows(dB, p)
    b = B.matvec(np.ones(B.n))
    pb = torch.from_numpy(b[ph.astype(np.int64)]).cuda()   # (P b)_k = b[p[k]]
    plan_c = rsai.build(C, **C1)
    x, it, rel = plan_c.bicgstab(pb)
    xh = x.cpu().numpy()
    res = np.linalg.norm(b - B.matvec(xh)) / np.linalg.norm(b)
    plan_b = rsai.build(dB, **C1)
    _, it_b, rel_b = plan_b.bicgstab(torch.from_numpy(b).cuda())
    print(f"BiCGStab iterations: permuted {it} (relres {rel:.2e}), unpermuted {it_b} (relres {rel_b:.2e})",
          flush=True)
    assert 0 < it <= 1000 and rel < 1e-8 and res < 1e-7
