"""The autotuner's success path and the tuning table applied through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen
from tests.parity import compare

pytestmark = pytest.mark.gpu
C1 = dict(c=3, lmax=8, eps=0.4, tol=1e-3)


def test_autotune_success_path():
    """rsai_autotune on a small matrix times all 28 schedule combinations (tier0,
    refill, route, the first tier's hash factor, the last register tier) and points
    at the fastest; builds with the fastest and the slowest choice both meet the
    parity bar against the oracle (schedules change speed, not results)."""
    import paper_1503_04500_amd.rsai as rsai
    from paper_1503_04500_amd import tune
    H = gen.cd2d(48, seed=2)
    A = rsai.Matrix.from_host(H, "cuda:0")
    r = tune.autotune(A, reps=1, validate=2, **C1)
    ch = r["choices"]
    assert len(ch) == 28
    assert r["best"]["ms"] == min(c["ms"] for c in ch) and all(c["ms"] > 0 for c in ch)
    keys = {tuple(c[k] for k in tune.KEYS) for c in ch}
    assert len(keys) == 28
    assert {c["t0_hash"] for c in ch} == {2, 4} and {c["last_tier"] for c in ch} == {1, 2}
    ref = oracle.rsai(H, **C1)
    worst = max(ch, key=lambda c: c["ms"])
    for c in (r["best"], worst):
        plan = rsai.build(A, tune_table=[], **C1, **{k: c[k] for k in tune.KEYS})
        assert plan.schedule() == {k: c[k] for k in tune.KEYS}
        cp, ri, va = (t.cpu().numpy() for t in plan.export())
        st = {k: v.cpu().numpy() for k, v in plan.stats().items()}
        compare(H, dict(colptr=cp, rowidx=ri, val=va, **st), ref, label=f"schedule {c}")


def test_tune_table_through_the_c_abi():
    """A table handed to rsai_build in rsai_params sets the schedule fields left at -1
    from the first matching entry (the library reads the longest column on the
    device); fields given explicitly win; no match keeps the defaults."""
    import paper_1503_04500_amd.rsai as rsai
    H = gen.cd2d(64, seed=1)       # mean column length 4.94, longest 5, n = 4096
    A = rsai.Matrix.from_host(H, "cuda:0")
    table = [dict(len_lo=1.0, len_hi=3.0, maxlen_lo=1, maxlen_hi=100, n_lo=1, n_hi=10**7, tier0=2, refill=0,
                  route=0, t0_hash=2, last_tier=2),      # mean length outside
             dict(len_lo=4.0, len_hi=6.0, maxlen_lo=5, maxlen_hi=6, n_lo=1000, n_hi=5000, tier0=0, refill=0,
                  route=0, t0_hash=4, last_tier=1),
             dict(len_lo=4.0, len_hi=6.0, maxlen_lo=1, maxlen_hi=100, n_lo=1, n_hi=10**7, tier0=1, refill=1,
                  route=1, t0_hash=2, last_tier=2)]
    p = rsai.build(A, tune_table=table, **C1)
    assert p.schedule() == dict(tier0=0, refill=0, route=0, t0_hash=4, last_tier=1)
    p2 = rsai.build(A, tune_table=table, refill=1, **C1)
    assert p2.schedule()["refill"] == 1 and p2.schedule()["t0_hash"] == 4
    p3 = rsai.build(A, tune_table=table[:1], **C1)
    assert p3.schedule() == dict(tier0=0, refill=1, route=1, t0_hash=2, last_tier=2)
    # a matrix whose longest column the host does not know: the library reads it
    Ad = rsai.Matrix(A.colptr, A.rowidx, A.val)
    assert Ad._max_col_len is None
    assert rsai.build(Ad, tune_table=table, **C1).schedule() == p.schedule()
    # the eps ranges of an entry
    te = [dict(table[2], eps_lo=0.3, eps_hi=1.0, tier0=0, last_tier=1),
          dict(table[2], eps_lo=0.0, eps_hi=0.3, tier0=1, last_tier=2)]
    assert rsai.build(A, tune_table=te, **C1).schedule()["last_tier"] == 1
    assert rsai.build(A, tune_table=te, **dict(C1, eps=0.2)).schedule()["tier0"] == 1
    ref = oracle.rsai(H, **C1)
    cp, ri, va = (t.cpu().numpy() for t in p.export())
    st = {k: v.cpu().numpy() for k, v in p.stats().items()}
    compare(H, dict(colptr=cp, rowidx=ri, val=va, **st), ref, label="tuned schedule")
