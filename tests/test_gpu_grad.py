"""GPU adjoint (rsai_backward) and the autograd loss vs the oracle's adjoint, and
y = M x (rsai_apply) vs the oracle's M."""
import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen
from tests.parity import compare_grad, run_gpu

pytestmark = pytest.mark.gpu
C1 = dict(c=3, lmax=8, eps=0.4, tol=1e-3)


def _oracle_grad(A, Mcp, Mri, b):
    mval, _ = oracle.fixed_pattern(A, Mcp, Mri)
    Mcsc = gen.CSC(A.n, Mcp, Mri, mval)
    u = Mcsc.matvec(b)
    s = A.matvec(u) - b
    ats = np.zeros(A.n)
    ce = A.col_of_entry()
    np.add.at(ats, ce, A.val * s[A.rowidx])
    gM = 2.0 * b[Mcsc.col_of_entry()] * ats[Mri]
    dA = oracle.backward(A, Mcp, Mri, mval, gM, w_frob=1.0)
    dA += 2.0 * s[A.rowidx] * u[ce]
    return dA, gM


@pytest.mark.parametrize("name,keep", [("c1", False), ("cd3d20", False), ("c1", True), ("cd3d20", True),
                                       ("cd3d20", "tiny"), ("cd3d12", True), ("powerlaw", True),
                                       ("denserows", True), ("cd3d12eps", True)])
def test_backward_kernel_vs_oracle(name, keep):
    """Refactorising adjoint, adjoint on the kept R factors, and a factor budget too
    small for all columns (both kernels in one call); with kept factors the |I_k|
    limit of the refactorising kernel does not apply (3D corner columns reach
    |I| = 71, power-law columns |I| = 232)."""
    import torch
    A = {"c1": gen.c1, "cd3d20": lambda: gen.cd3d(20, seed=1), "cd3d12": lambda: gen.cd3d(12, seed=3),
         "powerlaw": lambda: gen.powerlaw(3000, seed=11, lmax=20), "denserows": lambda: gen.dense_rows(64, 16, 48),
         "cd3d12eps": lambda: gen.cd3d(12, seed=3)}[name]()
    kw = {"powerlaw": dict(C1, lmax=2), "cd3d12eps": dict(C1, lmax=5, eps=0.1)}.get(name, C1)
    ref = oracle.rsai(A, **kw)
    fk = {} if keep is False else (dict(keep_factors=True, factor_budget_bytes=8 * 20000) if keep == "tiny"
                                   else dict(keep_factors=True))
    gpu = run_gpu(A, **kw, **fk)
    b = np.random.default_rng(0).standard_normal(A.n)
    want, gM = _oracle_grad(A, ref["colptr"], ref["rowidx"], b)
    assert np.array_equal(gpu["rowidx"], ref["rowidx"])
    # the adjoint part alone, through the C ABI, vs the oracle's adjoint on the GPU's M
    dA = torch.zeros(A.nnz, dtype=torch.float64, device="cuda:0")
    gpu["plan"].backward(torch.from_numpy(gM).cuda(), 1.0, dA)
    only, scale = oracle.backward(A, gpu["colptr"], gpu["rowidx"], gpu["val"], gM, w_frob=1.0, scale=True)
    got = dA.cpu().numpy()
    r = compare_grad(got, only, scale, label=f"{name}/{keep}")
    print(f"{name}/{keep}: max |gpu - oracle| / scale = {r:.2e}")


@pytest.mark.parametrize("name,fk", [
    ("denserows", dict(keep_factors=False)),
    ("cd3d12", dict(keep_factors=False)),
    ("powerlaw", dict(keep_factors=True, factor_budget_bytes=8)),
    ("powerlaw", dict(keep_factors=False)),
    ("denserows", dict(keep_factors=True, factor_budget_bytes=8)),
])
def test_backward_recomputes_large_columns(name, fk):
    """Columns without a kept factor that exceed the refactorising kernel's block
    (|J_k| > 32: dense-row columns; |I_k| > 64: 3D corner and power-law columns) get
    their factor recomputed (Cholesky of A_k^T A_k from sparse column products) and
    are differentiated on it: no RSAI_E_CAP, and entry-by-entry parity with the oracle's
    adjoint. factor_budget_bytes = 8 keeps no factor at all."""
    import torch
    A = {"denserows": lambda: gen.dense_rows(64, 16, 48), "cd3d12": lambda: gen.cd3d(12, seed=3),
         "powerlaw": lambda: gen.powerlaw(3000, seed=11, lmax=60)}[name]()
    kw = dict(C1, lmax=3) if name == "powerlaw" else C1
    gpu = run_gpu(A, **kw, **fk)
    nJ, nI = np.diff(gpu["colptr"]), gpu["nI"]
    big = (nJ > 32) | (nI > 64)
    assert big.sum() > 3, (int((nJ > 32).sum()), int((nI > 64).sum()))
    gM = np.sin(np.arange(gpu["val"].size, dtype=np.float64))
    dA = torch.zeros(A.nnz, dtype=torch.float64, device="cuda:0")
    gpu["plan"].backward(torch.from_numpy(gM).cuda(), 1.0, dA)
    want, scale = oracle.backward(A, gpu["colptr"], gpu["rowidx"], gpu["val"], gM, w_frob=1.0, scale=True)
    r = compare_grad(dA.cpu().numpy(), want, scale, label=f"{name}/{fk}")
    print(f"{name} {fk}: {int(big.sum())} large columns, max |gpu - oracle| / scale = {r:.2e}")


@pytest.mark.parametrize("name,fk", [("cd3d20", dict(keep_factors=True)), ("cd3d20", dict(keep_factors=False)),
                                     ("powerlaw", dict(keep_factors=True, factor_budget_bytes=8)),
                                     ("denserows", dict(keep_factors=True))])
def test_backward_deterministic_mode(name, fk):
    """deterministic = 1: every entry's contributions are added in column order after a
    sort, so two adjoint calls give bitwise-equal gradients; still entry-by-entry equal
    to the oracle's adjoint within the parity bar."""
    import torch
    A = {"cd3d20": lambda: gen.cd3d(20, seed=1), "powerlaw": lambda: gen.powerlaw(3000, seed=11, lmax=60),
         "denserows": lambda: gen.dense_rows(64, 16, 48)}[name]()
    kw = dict(C1, lmax=3) if name == "powerlaw" else C1
    gpu = run_gpu(A, **kw, **fk, deterministic=True)
    gM = np.cos(np.arange(gpu["val"].size, dtype=np.float64))
    outs = []
    for _ in range(3):
        dA = torch.zeros(A.nnz, dtype=torch.float64, device="cuda:0")
        gpu["plan"].backward(torch.from_numpy(gM).cuda(), 0.5, dA)
        outs.append(dA.cpu().numpy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:]), "fixed-order adjoint not repeatable"
    want, scale = oracle.backward(A, gpu["colptr"], gpu["rowidx"], gpu["val"], gM, w_frob=0.5, scale=True)
    compare_grad(outs[0], want, scale, label=f"det {name}")


def test_autograd_loss_gradient_c1():
    import torch
    from paper_1503_04500_amd import autograd as ag
    import paper_1503_04500_amd.rsai as rsai
    A = gen.c1()
    ref = oracle.rsai(A, **C1)
    b = np.random.default_rng(0).standard_normal(A.n)
    want, _ = _oracle_grad(A, ref["colptr"], ref["rowidx"], b)
    dA = rsai.Matrix.from_host(A, "cuda:0")
    val = dA.val.clone().requires_grad_(True)
    L = ag.rsai_loss(dA, val, torch.from_numpy(b).cuda(), **C1)
    L.backward()
    got = val.grad.cpu().numpy()
    assert np.allclose(got, want, rtol=1e-8, atol=1e-10 * np.abs(want).max())
    # the loss value
    mval, rn = oracle.fixed_pattern(A, ref["colptr"], ref["rowidx"])
    u = gen.CSC(A.n, ref["colptr"], ref["rowidx"], mval).matvec(b)
    s = A.matvec(u) - b
    assert abs(L.item() - (np.sum(rn ** 2) + s @ s)) <= 1e-9 * abs(L.item())


def test_autograd_vs_central_fd_c1():
    """Gradient within 1e-6 of central finite differences (step 1e-6) of the loss
    evaluated by the GPU path with the pattern fixed."""
    import torch
    from paper_1503_04500_amd import autograd as ag
    import paper_1503_04500_amd.rsai as rsai
    A = gen.c1()
    b = torch.from_numpy(np.random.default_rng(0).standard_normal(A.n)).cuda()
    dA = rsai.Matrix.from_host(A, "cuda:0")
    val = dA.val.clone().requires_grad_(True)
    L = ag.rsai_loss(dA, val, b, **C1)
    L.backward()
    g = val.grad.cpu().numpy()
    ref = oracle.rsai(A, **C1)
    Mcp, Mri = ref["colptr"], ref["rowidx"]
    bn = b.cpu().numpy()

    def loss_fixed(v):
        Av = A.with_values(v)
        mval, rn = oracle.fixed_pattern(Av, Mcp, Mri)
        u = gen.CSC(A.n, Mcp, Mri, mval).matvec(bn)
        s = Av.matvec(u) - bn
        return float(np.sum(rn ** 2) + s @ s)

    rng = np.random.default_rng(3)
    h = 1e-6
    for e in rng.choice(A.nnz, 25, replace=False):
        vp = A.val.copy(); vp[e] += h
        vm = A.val.copy(); vm[e] -= h
        fd = (loss_fixed(vp) - loss_fixed(vm)) / (2 * h)
        assert abs(g[e] - fd) <= 1e-6 * max(1.0, abs(fd)), (e, g[e], fd)


def test_apply_matches_oracle_M():
    import torch
    A = gen.c1()
    ref = oracle.rsai(A, **C1)
    gpu = run_gpu(A, **C1)
    x = np.random.default_rng(1).standard_normal(A.n)
    y = gpu["plan"].apply(torch.from_numpy(x).cuda()).cpu().numpy()
    want = gen.CSC(A.n, ref["colptr"], ref["rowidx"], ref["val"]).matvec(x)
    assert np.allclose(y, want, rtol=1e-10, atol=1e-13)


def test_bicgstab_iterations_equal_c1():
    """Right-preconditioned BiCGStab (Section 5 protocol: x0 = 0, b = A*1, relative
    residual < 1e-8) takes the same number of iterations with the GPU's M as with
    the oracle's M on the 32x32 case, where the count is stable."""
    A = gen.c1()
    ref = oracle.rsai(A, **C1)
    gpu = run_gpu(A, **C1)
    b = A.matvec(np.ones(A.n))
    it_o, rel_o, _ = oracle.bicgstab(A, b, (ref["colptr"], ref["rowidx"], ref["val"]))
    it_g, rel_g, _ = oracle.bicgstab(A, b, (gpu["colptr"], gpu["rowidx"], gpu["val"]))
    assert it_o == it_g == 36 and rel_g < 1e-8


def test_bicgstab_iterations_within_rounding_ensemble():
    """On the 128x128 random-convection grid the BiCGStab count is chaotic: a 1e-13
    relative perturbation of the oracle's own M moves it by tens of iterations. The
    GPU's M must converge and its count must fall inside the spread of counts of the
    oracle's M perturbed at the size of the observed GPU/oracle difference."""
    A = gen.cd2d(128, seed=0)
    ref = oracle.rsai(A, **C1)
    gpu = run_gpu(A, **C1)
    assert np.array_equal(gpu["rowidx"], ref["rowidx"])
    b = A.matvec(np.ones(A.n))
    it_g, rel_g, _ = oracle.bicgstab(A, b, (gpu["colptr"], gpu["rowidx"], gpu["val"]))
    assert rel_g < 1e-8 and it_g <= 1000
    delta = max(np.max(np.abs(gpu["val"] - ref["val"]) / np.abs(ref["val"])), 1e-15)
    its = []
    for s in range(12):
        v = ref["val"] * (1 + delta * np.random.default_rng(s).standard_normal(ref["val"].size))
        its.append(oracle.bicgstab(A, b, (ref["colptr"], ref["rowidx"], v))[0])
    lo, hi = min(its), max(its)
    slack = max(5, (hi - lo) // 2)
    assert lo - slack <= it_g <= hi + slack, (it_g, its)


def test_batched_loss_gradient_equals_single_builds():
    """One batched build of several matrices (2D, 3D, power-law with |J_k| > 32 on
    kept factors) differentiated at once: the loss and every matrix's gradient equal
    those of the single-matrix builds (same kernels; the adjoint order of the FP64
    atomics may differ, hence the rounding tolerance)."""
    import torch
    import paper_1503_04500_amd.rsai as rsai
    from paper_1503_04500_amd import autograd as ag
    Hs = [gen.cd2d(30, seed=1), gen.cd3d(9, seed=2), gen.dense_rows(32, 8, 40), gen.powerlaw(2000, seed=4, lmax=30)]
    mats = [rsai.Matrix.from_host(h, "cuda:0") for h in Hs]
    bs = [torch.from_numpy(np.random.default_rng(20 + i).standard_normal(h.n)).cuda() for i, h in enumerate(Hs)]
    vals = [m.val.clone().requires_grad_(True) for m in mats]
    L = ag.rsai_loss_batched(mats, vals, bs, **C1)
    L.backward()
    tot = 0.0
    for m, v, b in zip(mats, vals, bs):
        v1 = m.val.clone().requires_grad_(True)
        Li = ag.rsai_loss(m, v1, b, **C1)
        Li.backward()
        tot += Li.item()
        err = (v.grad - v1.grad).abs().max().item() / v1.grad.abs().max().item()
        assert err <= 1e-11, err
    assert abs(L.item() - tot) <= 1e-12 * abs(tot)


@pytest.mark.parametrize("name", ["budget_below_one_record", "three_columns"])
def test_backward_edge_cases_vs_oracle(name):
    """Kept factors with a store smaller than one record (every wave's chunk is too
    short, so every column is refactorised), and a matrix with fewer columns than
    the GPU has XCDs (most workgroups of the adjoint get an empty column range)."""
    import torch
    if name == "budget_below_one_record":
        A = gen.c1()
        fk = dict(keep_factors=True, factor_budget_bytes=8)
    else:
        A = gen.from_coo(3, np.array([0, 1, 2, 0, 1]), np.array([0, 1, 2, 1, 2]), np.array([4.0, 3.0, 5.0, 1.0, -1.0]))
        fk = dict(keep_factors=True)
    gpu = run_gpu(A, **C1, **fk)
    gM = 1.0 / (1.0 + (np.arange(gpu["val"].size) % 7))
    dA = torch.zeros(A.nnz, dtype=torch.float64, device="cuda:0")
    gpu["plan"].backward(torch.from_numpy(gM).cuda(), 0.5, dA)
    want, scale = oracle.backward(A, gpu["colptr"], gpu["rowidx"], gpu["val"], gM, w_frob=0.5, scale=True)
    compare_grad(dA.cpu().numpy(), want, scale, label=name)


@pytest.mark.parametrize("keep", [True, False])
def test_backward_c4_full_size_entrywise(keep):
    """The 3D 64^3 configuration (n = 262144, nnz = 1,810,432) at its own size: the
    adjoint of the GPU's build (on kept factors, and refactorised), entry by entry
    against the oracle's adjoint on the same M, with w_frob = 1 and an upstream
    gradient on every entry of M."""
    import torch
    A = gen.c4()
    assert A.n == 262144 and A.nnz == 1810432
    fk = dict(keep_factors=True) if keep else dict(keep_factors=False)
    gpu = run_gpu(A, **C1, **fk)
    assert gpu["status"].max() == 0
    gM = np.cos(np.arange(gpu["val"].size, dtype=np.float64))
    dA = torch.zeros(A.nnz, dtype=torch.float64, device="cuda:0")
    gpu["plan"].backward(torch.from_numpy(gM).cuda(), 1.0, dA)
    want, scale = oracle.backward(A, gpu["colptr"], gpu["rowidx"], gpu["val"], gM, w_frob=1.0, scale=True)
    r = compare_grad(dA.cpu().numpy(), want, scale, label="cd3d64")
    print(f"cd3d64 keep={keep}: max |gpu - oracle| / scale = {r:.2e}")
