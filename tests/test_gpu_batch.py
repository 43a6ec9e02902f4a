"""Batched solve (many QPs with diagonal Q in one persistent launch) against
the oracle, instance by instance, through the C ABI."""

import json
import os
import time

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2602_23967_amd as P
from paper_2602_23967_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need the MI355X"
    return T


def _unbounded_lp():
    """LP with a free variable that no row touches and a negative cost: the
    problem is unbounded along e_0 (diagonal Q = 0 fits the batch path)."""
    q = I.tiny_lp(40)
    A = q.A.toarray()
    A[:, 0] = 0.0
    q.A = sp.csr_matrix(A)
    q.lb = q.lb.copy(); q.ub = q.ub.copy()
    q.lb[0], q.ub[0] = -np.inf, np.inf
    q.c = q.c.copy(); q.c[0] = -1.0
    q.b = q.A @ np.full(q.n, 1.0)
    q.name = "unbounded_lp"
    return q


@pytest.fixture(scope="module")
def mix():
    qs = [I.mpc(i) for i in range(20)]
    qs += [I.mpc(100, infeasible=True), I.mpc(101, infeasible=True)]
    # (a portfolio's budget row is longer than QP_BATCH_MAX_ROW: not batched)
    qs += [I.tiny_lp(3), _unbounded_lp()]
    # non-diagonal Q: the inner boxed-CG solve runs inside the workgroup
    qs += [I.random_small(0), I.random_small(1, n=300), I.mixed_bounds(0), I.tiny(3, n=6, m=3),
           I.contradictory_rows(0), I.unbounded_qp(0)]
    return qs


def test_batch_matches_oracle(torch, mix):
    print(f"launch of {len(mix)} instances", flush=True)
    with P.BatchSolver(mix) as bs:
        st, secs = bs.solve()
        res = [bs.result(i) for i in range(len(mix))]
    print(f"launch done in {secs:.2f} s", flush=True)
    for q, g in zip(mix, res):
        o = oracle.solve(q, max_iter=100000)
        assert g.status == o.status, (q.name, g.status_name, o.status_name)
        if o.status == oracle.OPTIMAL:
            k = oracle.kkt(q, g.x, g.y)
            assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6, (q.name, k)
            ref = oracle.solve(q, tol=1e-9, max_iter=400000)
            f, fr = g.info["primal_obj"], ref.info["primal_obj"]
            assert abs(f - fr) <= 1e-6 * (1 + abs(fr)), (q.name, f, fr)
            assert np.all(g.x >= q.lb) and np.all(g.x <= q.ub)
        elif o.status == oracle.PRIMAL_INFEASIBLE:
            assert np.abs(g.y).max() == pytest.approx(1.0)
        elif o.status == oracle.DUAL_INFEASIBLE:
            d = g.x
            assert np.abs(d).max() == pytest.approx(1.0) and q.c @ d < 0
            assert np.abs(q.A @ d).max() <= 1e-8
    assert list(st) == [r.status for r in res]


def test_batch_iterates_match_oracle(torch):
    """Each instance's iterates after 150 iterations (checks every 5, so
    several restarts) equal the oracle's up to rounding order, in FP64: the
    persistent kernel runs the same steps and decisions per instance."""
    qs = [I.mpc(i) for i in range(6)] + [I.portfolio(1, n_assets=240, k_factors=3)]
    with P.BatchSolver(qs) as bs:
        st, _ = bs.solve(max_iter=150, check_every=5)
        res = [bs.result(i) for i in range(len(qs))]
    for q, g in zip(qs, res):
        o = oracle.solve(q, max_iter=150, check_every=5)
        assert g.status == o.status, q.name
        assert g.info["iterations"] == o.info["iterations"] and g.info["restarts"] == o.info["restarts"], q.name
        err = max(np.abs(g.x - o.x).max() / (1.0 + np.abs(o.x).max()),
                  np.abs(g.y - o.y).max() / (1.0 + np.abs(o.y).max()))
        print(f"{q.name}: restarts {g.info['restarts']}, max relative difference {err:.2e}", flush=True)
        assert err <= 1e-10, (q.name, err)


def test_batch_instance_times(torch):
    """Per-instance times of a persistent launch: the first instance is
    taken up at 0, every instance finishes after it was taken up, and the
    last finish lies within the launch's host-measured wall time."""
    qs = [I.mpc(i) for i in range(300)]
    with P.BatchSolver(qs) as bs:
        with pytest.raises(P.QPError):
            bs.times()   # before any solve
        a = time.perf_counter()
        st, secs = bs.solve()
        wall = time.perf_counter() - a
        t0, t1 = bs.times()
    print(f"300 instances: wall {wall * 1e3:.1f} ms, last finish {t1.max() * 1e3:.1f} ms, "
          f"median solve {np.median(t1 - t0) * 1e3:.2f} ms", flush=True)
    assert np.all(st == P.OPTIMAL)
    assert t0.min() == 0.0
    assert np.all(np.isfinite(t0)) and np.all(np.isfinite(t1)) and np.all(t1 > t0)
    assert t1.max() <= wall


def test_batch_alone_equals_in_the_mix(torch, mix):
    """An instance's result does not depend on the other instances of the
    launch (bitwise)."""
    picks = (3, 7, 21, 24, 26)
    with P.BatchSolver(mix) as bs:
        bs.solve()
        together = [bs.result(i) for i in picks]
    for i, g in zip(picks, together):
        with P.BatchSolver([mix[i]]) as one:
            one.solve()
            a = one.result(0)
        assert a.status == g.status and a.info["iterations"] == g.info["iterations"]
        assert np.array_equal(a.x, g.x) and np.array_equal(a.y, g.y)


def test_batch_deterministic_and_limits(torch):
    qs = [I.mpc(i) for i in range(30, 36)]
    with P.BatchSolver(qs) as bs:
        bs.solve()
        r1 = [bs.result(i) for i in range(len(qs))]
        bs.solve()
        r2 = [bs.result(i) for i in range(len(qs))]
        st0, _ = bs.solve(max_iter=0)
        assert np.all(st0 == P.ITERATION_LIMIT)
        st1, _ = bs.solve(max_iter=10)
        assert np.all(st1 == P.ITERATION_LIMIT)
    for a, b in zip(r1, r2):
        assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)


def test_batch_agrees_with_single_path(torch):
    """The one-instance path (separate kernels per step) and the batched
    path reach the same optimum."""
    q = I.mpc(7)
    with P.BatchSolver([q]) as bs:
        bs.solve()
        gb = bs.result(0)
    with P.Solver(q) as s:
        gs = s.solve()
    assert gb.status == gs.status == P.OPTIMAL
    assert gb.info["primal_obj"] == pytest.approx(gs.info["primal_obj"], rel=1e-6, abs=1e-9)
    assert np.abs(gb.x - gs.x).max() <= 1e-4


def test_batch_many_instances(torch):
    qs = [I.mpc(i) for i in range(200, 712)]
    with P.BatchSolver(qs) as bs:
        st, secs = bs.solve()
        print(f"512 MPC instances: {secs * 1e3:.1f} ms, {np.sum(st == P.OPTIMAL)} optimal")
        assert np.all(st == P.OPTIMAL)
        for i in (0, 255, 511):
            g = bs.result(i)
            k = oracle.kkt(qs[i], g.x, g.y)
            assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6


def test_mpc_batch_full_size_against_oracle(torch):
    """The 4096-instance MPC batch at full size, in mixed precision (its
    configuration) and FP64: every instance OPTIMAL with relative KKT <= 1e-6
    evaluated by the oracle on its returned point, and on the seeded 5 %
    sample the oracle solved at tol 1e-9 (stored:
    tests/golden/oracle_mpc_sample.json) the oracle's status and objective
    to 1e-6 (1 + |f|)."""
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_mpc_sample.json")) as f:
        gold = json.load(f)
    t = time.perf_counter()
    qs = [I.mpc(i) for i in range(4096)]
    print(f"generated 4096 MPC instances in {time.perf_counter() - t:.1f}s", flush=True)
    sample = {r["index"]: r for r in gold["results"]}
    with P.BatchSolver(qs) as bs:
        for prec in (P.PRECISION_MIXED, P.PRECISION_FP64):
            st, secs = bs.solve(precision=prec)
            print(f"precision {prec}: 4096 instances in {secs * 1e3:.1f} ms, "
                  f"{int(np.sum(st == P.OPTIMAL))} optimal", flush=True)
            assert np.all(st == P.OPTIMAL)
            worst_kkt = worst_obj = 0.0
            for i, q in enumerate(qs):
                g = bs.result(i)
                k = oracle.kkt(q, g.x, g.y)
                worst_kkt = max(worst_kkt, k["r_primal"], k["r_dual"], k["r_gap"])
                assert np.all(g.x >= q.lb) and np.all(g.x <= q.ub), q.name
                if i in sample:
                    r = sample[i]
                    assert r["instance"] == q.name and g.status == r["status"], (q.name, r["status_name"])
                    err = abs(g.info["primal_obj"] - r["primal_obj"]) / (1 + abs(r["primal_obj"]))
                    worst_obj = max(worst_obj, err)
            print(f"precision {prec}: worst relative KKT {worst_kkt:.2e} over 4096 instances; worst objective "
                  f"error {worst_obj:.2e} over the {len(sample)}-instance oracle sample", flush=True)
            assert worst_kkt <= 1e-6
            assert worst_obj <= 1e-6


def test_batch_general_q_matches_single_path(torch):
    q = I.random_small(2)
    with P.BatchSolver([q]) as bs:
        bs.solve()
        gb = bs.result(0)
    with P.Solver(q) as s:
        gs = s.solve()
    assert gb.status == gs.status == P.OPTIMAL
    assert gb.info["inner_iterations"] > 0
    assert gb.info["primal_obj"] == pytest.approx(gs.info["primal_obj"], rel=1e-6)


@pytest.fixture(scope="module")
def sched_mix():
    qs = [I.mpc(i) for i in range(40, 46)]
    qs += [I.random_small(3, n=300), I.mpc(102, infeasible=True), I.tiny_lp(5)]
    ref = [oracle.solve(q, max_iter=100000) for q in qs]
    return qs, ref


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_batch_every_schedule_matches_oracle(torch, sched_mix, precision):
    """Every compiled launch shape in both queue orders: the order changes
    no bit; each shape gives the oracle's status, a 1e-6 KKT point and the
    oracle's objective."""
    qs, ref = sched_mix
    params = P.qp_params_default(precision=precision)
    with P.BatchSolver(qs) as bs:
        for shape in range(P.qp_batch_num_shapes()):
            res = {}
            for order in (0, 1):
                bs.set_schedule(shape, order)
                assert bs.schedule() == (shape, order)
                bs.solve(params)
                res[order] = [bs.result(i) for i in range(len(qs))]
            print(f"shape {shape} {P.qp_batch_shape_info(shape)}: "
                  f"iterations {[r.info['iterations'] for r in res[0]]}", flush=True)
            for a, b in zip(res[0], res[1]):
                assert a.status == b.status and a.info["iterations"] == b.info["iterations"]
                assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
            for q, g, o in zip(qs, res[0], ref):
                assert g.status == o.status, (shape, q.name, g.status_name, o.status_name)
                if o.status == oracle.OPTIMAL:
                    k = oracle.kkt(q, g.x, g.y)
                    assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6, (shape, q.name, k)
                    assert g.info["primal_obj"] == pytest.approx(o.info["primal_obj"], rel=1e-6, abs=1e-6)


def test_batch_tune_picks_fastest_and_caches(torch, tmp_path):
    qs = [I.mpc(i) for i in range(500, 564)]
    cache = str(tmp_path / "schedules.json")
    ns = P.qp_batch_num_shapes()
    with P.BatchSolver(qs) as bs:
        e = bs.tune(cache=cache)
        print(f"tuned: shape {e['shape']} ({e['threads']} threads, {e['lds']} LDS doubles), "
              f"order {e['order']}; seconds {[round(s * 1e3, 1) for s in e['seconds']]} ms", flush=True)
        assert not e["cached"] and len(e["seconds"]) == 2 * ns
        assert all(s > 0 for s in e["seconds"])
        assert e["seconds"][2 * e["shape"] + e["order"]] == min(e["seconds"])
        assert bs.schedule() == (e["shape"], e["order"])
        st, _ = P.qp_batch_statuses(bs.h, len(qs))
        assert np.all(st == P.OPTIMAL)
        g = bs.result(3)
        k = oracle.kkt(qs[3], g.x, g.y)
        assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6
    with P.BatchSolver(qs) as bs2:
        e2 = bs2.tune(cache=cache)
        assert e2["cached"] and (e2["shape"], e2["order"]) == (e["shape"], e["order"])
        assert bs2.schedule() == (e["shape"], e["order"])


def test_batch_bound_storage_gives_the_same_bits(torch, monkeypatch):
    """The batch's box as byte classes (MPC: two (l, u) pairs) or as arrays:
    the same bits."""
    qs = [I.mpc(i) for i in range(50, 56)] + [I.mpc(103, infeasible=True), I.tiny_lp(7)]
    params = P.qp_params_default(precision=P.PRECISION_MIXED)

    def run():
        with P.BatchSolver(qs) as bs:
            bs.solve(params)
            return [bs.result(i) for i in range(len(qs))]

    a = run()
    monkeypatch.setenv("PDHCG_BOUND_STORAGE", "arrays")
    b = run()
    for q, g, h in zip(qs, a, b):
        assert g.status == h.status and g.info["iterations"] == h.info["iterations"], q.name
        assert np.array_equal(g.x, h.x) and np.array_equal(g.y, h.y), q.name


def _wide_separable(n=70000, m=60, per_row=120, seed=7):
    """A diagonal-Q QP with more than 65536 variables (short rows and
    columns, so it fits the batched kernel): a batch holding it takes the
    32-bit column indices."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(m):
        cj = np.sort(rng.choice(n, size=per_row, replace=False))
        rows += [i] * per_row
        cols += list(cj)
    A = sp.csr_matrix((rng.normal(size=len(rows)), (rows, cols)), shape=(m, n))
    A.sort_indices()
    x0 = rng.uniform(-0.5, 0.5, size=n)
    Q = sp.diags(rng.uniform(0.1, 1.0, size=n)).tocsr()
    sense = np.array([ord("E")] * (m // 2) + [ord("G")] * (m - m // 2), dtype=np.uint8)
    b = A @ x0
    return I.QP(n=n, m=m, Q=Q, A=A, c=rng.normal(size=n), b=b, sense=sense.tobytes(),
                lb=np.full(n, -1.0), ub=np.full(n, 1.0), name="wide_separable")


def test_batch_wide_instance_uses_32bit_columns(torch):
    """A batch with an instance of more than 65536 variables runs the
    products on 32-bit column indices; results still match the oracle, and
    a small instance in it gets the result it gets in a 16-bit batch up to
    the last bits of its reductions."""
    wide = _wide_separable()
    small = I.mpc(9)
    with P.BatchSolver([wide, small]) as bs:
        bs.solve()
        gw, gs = bs.result(0), bs.result(1)
    ow = oracle.solve(wide)
    assert gw.status == ow.status == P.OPTIMAL
    k = oracle.kkt(wide, gw.x, gw.y)
    assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6, k
    assert gw.info["primal_obj"] == pytest.approx(ow.info["primal_obj"], rel=1e-6, abs=1e-6)
    with P.BatchSolver([small]) as bs:
        bs.solve()
        a = bs.result(0)
    assert gs.status == a.status == P.OPTIMAL
    assert gs.info["iterations"] == a.info["iterations"]
    assert np.array_equal(gs.x, a.x) and np.array_equal(gs.y, a.y)
