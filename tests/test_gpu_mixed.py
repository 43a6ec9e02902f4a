"""Mixed precision (FP32 bulk products, FP64 iterates, checks and
certificates) against the FP64 oracle, single-problem and batched paths.

Every mixed result must carry the oracle's status and reach the relative KKT
tolerance evaluated in FP64 by the oracle from the returned (x, y); each test
prints the result's error against an FP64 reference solve."""

import json
import os

import numpy as np
import pytest

import oracle
import paper_2602_23967_amd as P
from paper_2602_23967_amd import instances as I

pytestmark = pytest.mark.gpu

MIXED = P.PRECISION_MIXED
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need the MI355X"
    return T


def _kkt_max(q, x, y):
    k = oracle.kkt(q, x, y)
    return max(k["r_primal"], k["r_dual"], k["r_gap"])


def _report(tag, q, g, ref):
    f, fr = g.info["primal_obj"], ref.info["primal_obj"]
    ferr = abs(f - fr) / (1 + abs(fr))
    xerr = float(np.abs(g.x - ref.x).max())
    print(f"{tag} {q.name}: kkt={_kkt_max(q, g.x, g.y):.2e} obj_err={ferr:.2e} x_err={xerr:.2e} "
          f"iters={g.info['iterations']}")
    return ferr, xerr


@pytest.mark.parametrize("make", [
    lambda: I.portfolio(1, n_assets=20000, k_factors=100),
    lambda: I.random_small(0),
    lambda: I.random_small(4, n=300),
    lambda: I.mixed_bounds(1),
    lambda: I.tiny_lp(2),
])
def test_mixed_single_matches_oracle(torch, make):
    q = make()
    with P.Solver(q) as s:
        g = s.solve(precision=MIXED)
    assert g.info["precision"] == MIXED
    o = oracle.solve(q, max_iter=400000)
    assert g.status == o.status == P.OPTIMAL, (g.status_name, o.status_name)
    assert _kkt_max(q, g.x, g.y) <= 1e-6
    assert np.all(g.x >= q.lb) and np.all(g.x <= q.ub)
    ref = oracle.solve(q, tol=1e-9, max_iter=400000)
    ferr, _ = _report("mixed", q, g, ref)
    assert ferr <= 1e-6


@pytest.mark.parametrize("make", ["contradictory", "box", "random_small"])
def test_mixed_primal_infeasible(torch, make):
    q = {"contradictory": lambda: I.contradictory_rows(1), "box": lambda: I.box_infeasible_rows(1),
         "random_small": lambda: I.random_small(2, infeasible=True)}[make]()
    with P.Solver(q) as s:
        g = s.solve(precision=MIXED, max_iter=20000)
    o = oracle.solve(q, max_iter=20000)
    assert g.status == o.status == P.PRIMAL_INFEASIBLE
    assert np.abs(g.y).max() == pytest.approx(1.0)


def test_mixed_unbounded(torch):
    q = I.unbounded_qp(1)
    with P.Solver(q) as s:
        g = s.solve(precision=MIXED, max_iter=20000)
    o = oracle.solve(q, max_iter=20000)
    assert g.status == o.status == P.DUAL_INFEASIBLE
    d = g.x
    assert np.abs(d).max() == pytest.approx(1.0) and q.c @ d < 0


def test_mixed_is_deterministic_and_fp64_unchanged(torch):
    """Two mixed solves agree bitwise; an FP64 solve after a mixed one on the
    same handle is bitwise the FP64 solve of a fresh handle."""
    q = I.random_small(1)
    with P.Solver(q) as s:
        a = s.solve(precision=MIXED)
        b = s.solve(precision=MIXED)
        c = s.solve()
    with P.Solver(q) as s2:
        d = s2.solve()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
    assert c.info["precision"] == P.PRECISION_FP64
    assert np.array_equal(c.x, d.x) and np.array_equal(c.y, d.y)


def test_invalid_precision_rejected(torch):
    q = I.tiny(0)
    with P.Solver(q) as s:
        with pytest.raises(P.QPError) as e:
            s.solve(precision=2)
        assert e.value.code == P.ERR_INVALID_ARG


def test_mixed_portfolio_full_size(torch):
    """The 200k-asset, 1000-factor portfolio in FP64 and in mixed precision:
    each carries the oracle's status, reaches relative KKT <= 1e-6 evaluated
    by the oracle, and matches the objective of the oracle run at tol 1e-9
    (stored: tests/golden/oracle_portfolio_200k.json) to 1e-6 (1 + |f|)."""
    q = I.portfolio(0)
    gold = json.load(open(os.path.join(GOLDEN, "oracle_portfolio_200k.json")))["result"]
    assert (gold["n"], gold["m"], gold["nnz_A"]) == (q.n, q.m, q.nnz_A)
    with P.Solver(q) as s:
        g64 = s.solve()
        g32 = s.solve(precision=MIXED)
    fr = gold["primal_obj"]
    for tag, g in (("fp64", g64), ("mixed", g32)):
        f = g.info["primal_obj"]
        err = abs(f - fr) / (1 + abs(fr))
        print(f"portfolio 200k {tag}: {g.info['iterations']} it {g.info['solve_seconds'] * 1e3:.1f} ms; "
              f"kkt {_kkt_max(q, g.x, g.y):.2e}; objective error vs the oracle at tol 1e-9 {err:.2e}")
        assert g.status == gold["status"] == P.OPTIMAL
        assert _kkt_max(q, g.x, g.y) <= 1e-6
        assert np.all(g.x >= q.lb) and np.all(g.x <= q.ub)
        assert err <= 1e-6


def test_mixed_batch_matches_oracle(torch):
    qs = [I.mpc(i) for i in range(40, 52)] + [I.mpc(120, infeasible=True)]
    qs += [I.random_small(5, n=300), I.tiny_lp(4), I.contradictory_rows(2)]
    with P.BatchSolver(qs) as bs:
        st, _ = bs.solve(precision=MIXED)
        res = [bs.result(i) for i in range(len(qs))]
    worst = 0.0
    for q, g in zip(qs, res):
        o = oracle.solve(q, max_iter=100000)
        assert g.status == o.status, (q.name, g.status_name, o.status_name)
        if o.status == P.OPTIMAL:
            assert _kkt_max(q, g.x, g.y) <= 1e-6, q.name
            ref = oracle.solve(q, tol=1e-9, max_iter=400000)
            ferr, _ = _report("batch-mixed", q, g, ref)
            worst = max(worst, ferr)
            assert ferr <= 1e-6
        elif o.status == P.PRIMAL_INFEASIBLE:
            assert np.abs(g.y).max() == pytest.approx(1.0)
    print(f"worst objective error {worst:.2e}")


def test_mixed_batch_alone_equals_in_the_mix(torch):
    qs = [I.mpc(i) for i in range(60, 70)]
    with P.BatchSolver(qs) as bs:
        bs.solve(precision=MIXED)
        together = bs.result(4)
    with P.BatchSolver([qs[4]]) as one:
        one.solve(precision=MIXED)
        alone = one.result(0)
    assert alone.status == together.status == P.OPTIMAL
    assert np.array_equal(alone.x, together.x) and np.array_equal(alone.y, together.y)
