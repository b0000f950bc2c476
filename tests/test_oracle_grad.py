"""Pins of the oracle's fixed-pattern adjoint (gradients w.r.t. the values of A).

Loss (pattern of M fixed from a forward RSAI pass, values from the LS solves (2.3)):
    L(A) = sum_k ||A m_k - e_k||^2 + ||A M b - b||^2.
The adjoint is checked against central finite differences (step 1e-6), against
torch CPU autograd through the normal equations on a tiny case, and against the
envelope identity (the part of sum_k ||r_k||^2 that flows through M vanishes,
since A_k^T r_k = 0).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1503_04500_amd import gen


def loss(A, Mcp, Mri, b):
    mval, rn = oracle.fixed_pattern(A, Mcp, Mri)
    Mcsc = gen.CSC(A.n, Mcp, Mri, mval)
    u = Mcsc.matvec(b)
    s = A.matvec(u) - b
    return float(np.sum(rn ** 2) + s @ s)


def grad(A, Mcp, Mri, b):
    mval, _ = oracle.fixed_pattern(A, Mcp, Mri)
    Mcsc = gen.CSC(A.n, Mcp, Mri, mval)
    u = Mcsc.matvec(b)
    s = A.matvec(u) - b
    # A^T s
    ats = np.zeros(A.n)
    ce = A.col_of_entry()
    np.add.at(ats, ce, A.val * s[A.rowidx])
    mce = Mcsc.col_of_entry()
    gM = 2.0 * b[mce] * ats[Mri]          # dL2/dm_jk = 2 b_k (A^T s)_j
    dA = oracle.backward(A, Mcp, Mri, mval, gM, w_frob=1.0)
    dA += 2.0 * s[A.rowidx] * u[ce]        # direct part of L2 at fixed M
    return dA


@pytest.fixture(scope="module")
def c1_case():
    A = gen.c1()
    R = oracle.rsai(A, c=3, lmax=8, eps=0.4, tol=1e-3)
    b = np.random.default_rng(0).standard_normal(A.n)
    return A, R["colptr"], R["rowidx"], b


def test_adjoint_vs_central_fd_c1(c1_case):
    A, Mcp, Mri, b = c1_case
    g = grad(A, Mcp, Mri, b)
    rng = np.random.default_rng(1)
    idx = rng.choice(A.nnz, 60, replace=False)
    h = 1e-6
    for e in idx:
        vp = A.val.copy(); vp[e] += h
        vm = A.val.copy(); vm[e] -= h
        fd = (loss(A.with_values(vp), Mcp, Mri, b) - loss(A.with_values(vm), Mcp, Mri, b)) / (2 * h)
        assert abs(g[e] - fd) <= 1e-6 * max(1.0, abs(fd)), (e, g[e], fd)


def test_adjoint_directional_fd_c1(c1_case):
    A, Mcp, Mri, b = c1_case
    g = grad(A, Mcp, Mri, b)
    rng = np.random.default_rng(2)
    for _ in range(3):
        d = rng.standard_normal(A.nnz)
        h = 1e-6
        fd = (loss(A.with_values(A.val + h * d), Mcp, Mri, b) -
              loss(A.with_values(A.val - h * d), Mcp, Mri, b)) / (2 * h)
        assert abs(g @ d - fd) <= 1e-6 * max(1.0, abs(fd))


def test_envelope_identity(c1_case):
    """Feeding g_k = 2 A_k^T r_k (the through-M part of sum ||r_k||^2) gives ~0."""
    A, Mcp, Mri, _ = c1_case
    mval, _ = oracle.fixed_pattern(A, Mcp, Mri)
    d = A.to_dense()
    gM = np.zeros_like(mval)
    for k in range(A.n):
        s, e = Mcp[k], Mcp[k + 1]
        J = Mri[s:e]
        r = d[:, J] @ mval[s:e] - (np.arange(A.n) == k)
        gM[s:e] = 2.0 * d[:, J].T @ r
    assert np.abs(gM).max() < 1e-12
    dA = oracle.backward(A, Mcp, Mri, mval, gM, w_frob=0.0)
    assert np.abs(dA).max() < 1e-10


def test_adjoint_vs_torch_autograd_tiny():
    """Tiny matrix: torch CPU float64 autograd through the normal equations."""
    A = gen.cd2d(4, seed=3)
    R = oracle.rsai(A, c=2, lmax=3, eps=0.2, tol=1e-3)
    Mcp, Mri = R["colptr"], R["rowidx"]
    b = np.random.default_rng(5).standard_normal(A.n)
    g = grad(A, Mcp, Mri, b)

    val = torch.tensor(A.val, dtype=torch.float64, requires_grad=True)
    rows = torch.tensor(A.rowidx.astype(np.int64))
    cols = torch.tensor(A.col_of_entry())
    Ad = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((rows, cols), val)
    Mfull = torch.zeros(A.n, A.n, dtype=torch.float64)
    L = torch.zeros((), dtype=torch.float64)
    cols_m = []
    for k in range(A.n):
        J = torch.tensor(Mri[Mcp[k]:Mcp[k + 1]].astype(np.int64))
        B = Ad[:, J]
        ek = torch.zeros(A.n, dtype=torch.float64); ek[k] = 1.0
        m = torch.linalg.solve(B.T @ B, B.T @ ek)
        L = L + torch.sum((B @ m - ek) ** 2)
        cols_m.append((J, m))
    for k, (J, m) in enumerate(cols_m):
        Mfull = Mfull.index_put((J, torch.full_like(J, k)), m)
    bt = torch.tensor(b)
    s = Ad @ (Mfull @ bt) - bt
    L = L + s @ s
    L.backward()
    assert np.allclose(val.grad.numpy(), g, rtol=1e-9, atol=1e-11)
    assert abs(L.item() - loss(A, Mcp, Mri, b)) < 1e-10
