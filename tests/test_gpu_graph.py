"""rsai_rebuild: the build's kernel sequence run again for new values of A, eagerly
and as a captured HIP graph; every replay equals a fresh build with those values."""
import numpy as np
import pytest

from paper_1503_04500_amd import gen

pytestmark = pytest.mark.gpu

KW = dict(c=3, lmax=8, eps=0.4, tol=1e-3, validate=2)


def _result(plan):
    cp, ri, va = (t.cpu().numpy() for t in plan.export())
    st = {k: v.cpu().numpy() for k, v in plan.stats().items()}
    return dict(colptr=cp, rowidx=ri, val=va, **st)


def _same(a, b, label):
    for key in ("colptr", "rowidx", "val", "loops", "nI", "nJ", "resnorm", "status"):
        assert np.array_equal(a[key], b[key]), f"{label}: {key}"


@pytest.mark.parametrize("sched,which", [("batched", "cd2d"), ("batched", "powerlaw"), ("plain", "cd2d")])
def test_rebuild_replays_match_fresh_builds(sched, which):
    import torch
    import paper_1503_04500_amd.rsai as rsai
    H = gen.cd2d(40, seed=3) if which == "cd2d" else gen.powerlaw(6000, seed=4, lmax=40)
    rng = np.random.default_rng(11)
    vals = [H.val] + [H.val * (1.0 + 0.05 * rng.standard_normal(H.nnz)) for _ in range(2)]
    # the plain schedule has one size class: fewer loops keep every column inside it
    kw = dict(KW, lmax=2) if sched == "plain" else KW
    # references: a fresh build per value set
    refs = []
    for v in vals:
        A = rsai.Matrix.from_host(H.with_values(v), "cuda:0")
        refs.append(_result(rsai.build(A, sched=sched, **kw)))
    assert not np.array_equal(refs[0]["val"], refs[1]["val"])
    A = rsai.Matrix.from_host(H, "cuda:0")
    plan = rsai.build(A, sched=sched, **kw)
    _same(_result(plan), refs[0], "initial")
    order = [1, 2, 0, 1, 1, 2]
    for step, i in enumerate(order):
        A.val.copy_(torch.from_numpy(vals[i]).to("cuda:0"))
        plan.rebuild(graph=(step % 3 != 2))
        got = _result(plan)
        _same(got, refs[i], f"replay {step} (values {i})")
        # eager work on the same stream between replays
        y = plan.apply(torch.ones(H.n, dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()


def test_batched_multi_matrix_graph_replay():
    """A plan of several matrices (2D, 3D, power-law) in one batched build, replayed
    as a captured graph with new values in every matrix: each replay equals a fresh
    batched build with those values, matrix by matrix, bit for bit."""
    import torch
    import paper_1503_04500_amd.rsai as rsai
    Hs = [gen.cd2d(40, seed=3), gen.cd3d(10, seed=2), gen.powerlaw(5000, seed=4, lmax=40)]
    rng = np.random.default_rng(21)
    vsets = [[H.val for H in Hs]] + [[H.val * (1.0 + 0.05 * rng.standard_normal(H.nnz)) for H in Hs]
                                     for _ in range(2)]

    def results(plan):
        out = []
        for i in range(len(Hs)):
            cp, ri, va = (t.cpu().numpy() for t in plan.export(i))
            st = {k: v.cpu().numpy() for k, v in plan.stats(i).items()}
            out.append(dict(colptr=cp, rowidx=ri, val=va, **st))
        return out

    refs = []
    for vs in vsets:
        ms = [rsai.Matrix.from_host(H.with_values(v), "cuda:0") for H, v in zip(Hs, vs)]
        refs.append(results(rsai.build_batched(ms, **KW)))
    mats = [rsai.Matrix.from_host(H, "cuda:0") for H in Hs]
    plan = rsai.build_batched(mats, **KW)
    for i, r in enumerate(results(plan)):
        _same(r, refs[0][i], f"initial matrix {i}")
    for step, j in enumerate([1, 2, 0, 2]):
        for m, v in zip(mats, vsets[j]):
            m.val.copy_(torch.from_numpy(v).to("cuda:0"))
        plan.rebuild(graph=True)
        got = results(plan)
        for i in range(len(Hs)):
            _same(got[i], refs[j][i], f"replay {step} (values {j}) matrix {i}")
        y = plan.apply(torch.ones(Hs[0].n, dtype=torch.float64, device="cuda:0"), mat=0)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
