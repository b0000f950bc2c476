"""Pins of the oracle's work model and decision margins (no GPU).

The model flop count (Algorithm 1, step 7: the LS factor updated as J_k grows)
is the numerator of the benchmark's FP64 roofline, and the decision margins decide
which columns a rounding-level pattern divergence may be forgiven on. Both are
pinned here against hand counts (``tests/golden/flop_model_by_hand.json``), closed
forms of the same sums, a splitting identity and the leading-order Householder
costs; the margins against hand-built columns with exactly known values.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "flop_model_by_hand.json")))


def _new_reflectors(m, qlo, qn):
    """Closed form of sum_{j=qlo}^{qn-1} (m - j) (6 + 4 (qn - 1 - j)): with
    t = qn - 1 - j running over 0..p-1 (p = qn - qlo), m - j = (m - qn + 1) + t, so the
    sum is 6 [p a + p(p-1)/2] + 4 [a p(p-1)/2 + (p-1)p(2p-1)/6], a = m - qn + 1."""
    p = qn - qlo
    a = m - qn + 1
    s1 = p * a + Fraction(p * (p - 1), 2)
    s2 = a * Fraction(p * (p - 1), 2) + Fraction((p - 1) * p * (2 * p - 1), 6)
    return 6 * s1 + 4 * s2


def _closed(m0, m, qlo, qn):
    p = qn - qlo
    old = 4 * p * (qlo * m0 - Fraction(qlo * (qlo - 1), 2))  # sum_{j<qlo} 4 (m0 - j) p
    return old + _new_reflectors(m, qlo, qn) + qn * qn + 2 * (m - qn)


def test_model_matches_hand_counts():
    for case in GOLD["cases"]:
        if "m" in case:
            assert oracle.model_solve_flops(case["m0"], case["m"], case["qlo"], case["qn"]) == case["flops"], case
            if "terms" in case:
                t = case["terms"]
                tot = sum(sum(v) if isinstance(v, list) else v for v in t.values())
                assert tot == case["flops"], case  # the hand terms add up
        for s in case.get("solves", []):
            assert oracle.model_solve_flops(s["m0"], s["m"], s["qlo"], s["qn"]) == s["flops"], s


def test_model_matches_closed_form_sums():
    for m in (1, 2, 3, 5, 9, 21, 64, 200):
        for qn in range(1, min(m, 40) + 1):
            for qlo in sorted({0, 1, qn // 2, qn - 1}):
                for m0 in sorted({qlo, (qlo + m) // 2, m}):
                    if qlo == 0:
                        m0 = 0
                    got = oracle.model_solve_flops(m0, m, qlo, qn)
                    assert got == float(_closed(m0, m, qlo, qn)), (m0, m, qlo, qn)


def test_model_lmax0_is_8m_minus_1():
    """lmax = 0: one solve of |I_k| x 1 per column, 2m (norm) + 4m (Q^T e) + 1 (back
    substitution) + 2(m - 1) (residual norm) = 8m - 1, a function of |I_k| alone."""
    for A in (gen.c1(), gen.powerlaw(3000, seed=3), gen.cd3d(6)):
        ref = oracle.rsai(A, c=3, lmax=0, eps=0.4, drop=oracle.DROP_NONE)
        assert np.array_equal(ref["mflops"], 8.0 * ref["nI"] - 1.0)


def test_model_splitting_identity():
    """Without new rows (m0 = m), factoring the first qlo columns and then updating to
    qn costs what a from-scratch factor of all qn does, plus the first factor's own
    back substitution and residual norm."""
    for m in (4, 17, 50):
        for qn in range(2, min(m, 20) + 1):
            for qlo in range(1, qn):
                whole = oracle.model_solve_flops(0, m, 0, qn)
                first = oracle.model_solve_flops(0, m, 0, qlo)
                upd = oracle.model_solve_flops(m, m, qlo, qn)
                assert whole == first - qlo * qlo - 2 * (m - qlo) + upd, (m, qlo, qn)


def test_model_leading_order():
    """A from-scratch m x q solve approaches the textbook Householder cost
    2 m q^2 - (2/3) q^3 (factor) + 4 m q (Q^T e) as m, q grow; an update of p columns
    onto an m0 x q factor approaches 4 p (q m0 - q^2 / 2) + 2 (m - q) p^2 - (2/3) p^3
    + 4 (m - q) p."""
    for scale in (10, 100, 1000):
        m, q = 4 * scale, scale
        ref = 2 * m * q * q - (2.0 / 3.0) * q ** 3 + 4 * m * q
        got = oracle.model_solve_flops(0, m, 0, q)
        assert abs(got / ref - 1.0) < 3.0 / q
        m0, q0, p = 3 * scale, scale, scale
        m1 = m0 + scale
        ref = 4 * p * (q0 * m0 - q0 * q0 / 2.0) + 2 * (m1 - q0) * p * p - (2.0 / 3.0) * p ** 3 + 4 * (m1 - q0) * p
        got = oracle.model_solve_flops(m0, m1, q0, q0 + p)
        assert abs(got / ref - 1.0) < 3.0 / p


def test_model_per_column_worked_example():
    A = gen.c1()
    k = 10 + 32 * 10
    ref = oracle.rsai(A, c=3, lmax=8, eps=0.4, tol=1e-3, cols=[k])
    assert ref["loops"][0] == 1 and ref["ndrop"][0] == 0
    assert ref["mflops"][0] == GOLD["cases"][2]["flops"]


def test_model_per_column_two_by_two():
    A = gen.from_dense(np.array([[2.0, 1.0], [1.0, 2.0]]))
    r = oracle.rsai(A, c=1, lmax=1, eps=0.0, tol=0.35, cols=[0])
    assert r["ndrop"][0] == 1 and r["nJ"][0] == 1
    assert r["mflops"][0] == GOLD["cases"][3]["flops"]
    r = oracle.rsai(A, c=1, lmax=1, eps=0.0, tol=0.3, cols=[0])
    assert r["ndrop"][0] == 0 and r["nJ"][0] == 2
    assert r["mflops"][0] == GOLD["cases"][4]["flops"]


def _frac(d):
    return d["value_num"] / d["value_den"] if "value_num" in d else d["value"]


def test_sel_margin_worked_example():
    dm = GOLD["decision_margins"]
    A = gen.c1()
    k = 10 + 32 * 10
    r3 = oracle.rsai(A, c=3, lmax=8, eps=0.4, tol=1e-3, cols=[k])
    d = dm["c1_interior_c3_sel_margin"]
    assert abs(r3["sel_margin"][0] - d["value"]) <= d["atol"]
    r4 = oracle.rsai(A, c=4, lmax=8, eps=0.4, tol=1e-3, cols=[k])
    assert r4["sel_margin"][0] == 0.0
    A2 = gen.from_dense(np.array([[2.0, 1.0], [1.0, 2.0]]))
    r = oracle.rsai(A2, c=1, lmax=1, eps=0.0, tol=0.35, cols=[0])
    d = dm["two_by_two_sel_margin"]
    assert abs(r["sel_margin"][0] - _frac(d)) <= d["atol"]


def test_drop_margin_hand_built():
    dm = GOLD["decision_margins"]
    A2 = gen.from_dense(np.array([[2.0, 1.0], [1.0, 2.0]]))
    for tol, key in ((0.35, "two_by_two_tol035_drop_margin"), (0.3, "two_by_two_tol030_drop_margin")):
        r = oracle.rsai(A2, c=1, lmax=1, eps=0.0, tol=tol, cols=[0])
        d = dm[key]
        assert abs(r["drop_margin"][0] - _frac(d)) <= d["atol"], (tol, r["drop_margin"][0])
    D = gen.diagonal(np.array([4.0, 4.0, 4.0]))
    r = oracle.rsai(D, c=3, lmax=8, eps=0.4, tol=1e-3)
    d = dm["diagonal_4_drop_margin"]
    assert np.all(np.abs(r["drop_margin"] - d["value"]) <= d["atol"])


def test_margins_without_decisions_are_infinite():
    """No selection (lmax = 0) and no drop test (drop none) leave the margins at +inf."""
    r = oracle.rsai(gen.c1(), c=3, lmax=0, eps=0.4, drop=oracle.DROP_NONE)
    assert np.all(np.isinf(r["sel_margin"])) and np.all(np.isinf(r["drop_margin"]))


@pytest.mark.parametrize("c", [1, 3])
def test_sel_margin_is_the_selection_gap(c):
    """On random columns, sel_margin equals the gap recomputed from the residual the
    oracle's own loop-0 solution gives (one selection: lmax = 1)."""
    A = gen.powerlaw(400, seed=11)
    cols = np.arange(0, 400, 7)
    r = oracle.rsai(A, c=c, lmax=1, eps=0.0, drop=oracle.DROP_NONE, cols=cols)
    d = A.to_dense()
    for t, k in enumerate(cols):
        a = d[:, k]
        # loop 0 solution by least squares on the single column
        m0 = np.linalg.lstsq(a[:, None], np.eye(400)[:, k], rcond=None)[0][0]
        res = a * m0 - np.eye(400)[:, k]
        cand = np.sort(np.abs(res[res != 0.0]))[::-1]
        if cand.size <= c:
            assert np.isinf(r["sel_margin"][t])
            continue
        gap = cand[c - 1] - cand[c]
        assert abs(r["sel_margin"][t] - gap) <= 1e-12, (k, r["sel_margin"][t], gap)
