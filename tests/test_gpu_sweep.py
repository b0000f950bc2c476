"""Parameter sweeps (eps, c, dropping mode; the settings varied in Section 5) and
the dense-row regime of Section 4, GPU vs the oracle."""
import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen
from tests.parity import compare, run_gpu

pytestmark = pytest.mark.gpu
DROP = {"none": oracle.DROP_NONE, "fixed": oracle.DROP_FIXED, "adaptive": oracle.DROP_ADAPTIVE}


@pytest.mark.parametrize("eps,c,drop", [(0.2, 3, "fixed"), (0.3, 1, "fixed"), (0.5, 5, "fixed"),
                                        (0.3, 3, "adaptive"), (0.2, 2, "none"), (0.3, 5, "adaptive")])
def test_parameter_parity(eps, c, drop):
    """Full parity on a 48x48 random-convection grid across stopping criteria,
    numbers of dominant indices per loop and the three dropping modes (eps = 0.2
    reaches |J_k| = 58, past the register tiers)."""
    A = gen.cd2d(48, seed=3)
    ref = oracle.rsai(A, c=c, lmax=8, eps=eps, drop=DROP[drop], tol=1e-3)
    gpu = run_gpu(A, c=c, lmax=8, eps=eps, drop=drop, tol=1e-3)
    compare(A, gpu, ref, label=f"eps={eps} c={c} {drop}")


@pytest.mark.parametrize("N", [48, 128])
def test_eps01_parity(N):
    """eps = 0.1, the smallest of the paper's eps settings: every column runs to lmax on
    blocks of about 100 x 64 (on the 128x128 grid |J_k| reaches 68 before dropping,
    |I_k| 101), so nearly all columns finish in the workgroup classes. Full parity."""
    A = gen.cd2d(N, seed=3 if N == 48 else 0)
    ref = oracle.rsai(A, c=3, lmax=8, eps=0.1, drop=oracle.DROP_FIXED, tol=1e-3)
    gpu = run_gpu(A, c=3, lmax=8, eps=0.1, drop="fixed", tol=1e-3)
    s = compare(A, gpu, ref, label=f"eps=0.1 {N}x{N}")
    print(f"eps=0.1 {N}x{N}: nJ max {int(ref['nJ'].max())}, nJmax {int(ref['nJmax'].max())}, "
          f"nI max {int(ref['nI'].max())}, parity {s}", flush=True)


def test_smaller_eps_gives_denser_m_and_fewer_iterations():
    """The trend of the paper's eps experiments on a 128x128 grid: M gets denser as
    eps falls, and the device BiCGStab needs fewer iterations with it."""
    import torch
    A = gen.cd2d(128, seed=0)
    b = torch.from_numpy(A.matvec(np.ones(A.n))).cuda()
    nnz, its = [], []
    for eps in (0.5, 0.4, 0.3, 0.2):
        gpu = run_gpu(A, c=3, lmax=8, eps=eps, drop="fixed", tol=1e-3)
        nnz.append(int(gpu["colptr"][-1]))
        x, it, rel = gpu["plan"].bicgstab(b)
        assert 0 < it <= 1000 and rel < 1e-8
        its.append(it)
    assert all(a < b for a, b in zip(nnz, nnz[1:])), nnz
    assert its[-1] < its[0], its


def test_dense_rows_small_full_parity():
    """64x64 grid with 16 rows of 48 entries: columns that select a dense row pull
    its pattern into J_k (|J_k| up to 114 before dropping, 47 after; |I_k| up to
    480), so some solves run in the dense class beyond 64 columns."""
    A = gen.dense_rows(64, 16, 48)
    ref = oracle.rsai(A, c=3, lmax=8, eps=0.4, drop=oracle.DROP_FIXED, tol=1e-3)
    assert ref["nJ"].max() > 32 and ref["nJmax"].max() > 64
    gpu = run_gpu(A, c=3, lmax=8, eps=0.4, drop="fixed", tol=1e-3)
    compare(A, gpu, ref, label="dense-rows-64")


def test_dense_rows_512_full_parity():
    """The dense-row benchmark matrix (512x512 grid, 1024 rows of 32 entries) in
    full: about 400 columns end with |J_k| > 32, 177 pass 64 columns before dropping
    (up to 116)."""
    A = gen.dense_rows(512, 1024, 32)
    ref = oracle.rsai(A, c=3, lmax=8, eps=0.4, drop=oracle.DROP_FIXED, tol=1e-3)
    assert (ref["nJmax"] > 64).sum() > 100 and ref["nJmax"].max() <= 128
    gpu = run_gpu(A, c=3, lmax=8, eps=0.4, drop="fixed", tol=1e-3)
    s = compare(A, gpu, ref, label="dense-rows-512")
    print("dense rows 512", s)


def test_eps01_256_queue_capacity():
    """eps = 0.1 on a 256x256 grid sends about 48000 of the 65536 columns past the
    sparse-block class (their compressed blocks, with most rows shared, do not fit it)
    to the dense class: with the default queue capacity the build ends with RSAI_E_CAP
    and a message naming spill_capacity; with spill_capacity = n every column fits and a
    seeded sample of 1500 columns matches the oracle."""
    import paper_1503_04500_amd.rsai as rsai
    from tests.parity import subset
    A = gen.cd2d(256, seed=0)
    dA = rsai.Matrix.from_host(A, "cuda:0")
    with pytest.raises(rsai.RSAIError) as ei:
        rsai.build(dA, c=3, lmax=8, eps=0.1, tol=1e-3).nnz()
    assert ei.value.code == -6 and "spill_capacity" in str(ei.value)
    gpu = run_gpu(A, c=3, lmax=8, eps=0.1, drop="fixed", tol=1e-3, spill_capacity=A.n)
    cols = np.sort(np.random.default_rng(11).choice(A.n, 1500, replace=False))
    ref = oracle.rsai(A, c=3, lmax=8, eps=0.1, drop=oracle.DROP_FIXED, tol=1e-3, cols=cols)
    s = compare(A, subset(gpu, cols), ref, label="eps=0.1 256x256 sample", margin_tol=1e-14)
    print(f"eps=0.1 256x256 with spill_capacity=n: sample parity {s}", flush=True)
