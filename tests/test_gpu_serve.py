"""Request server (continuous batching) through the C ABI: every request's
result is the one the same problem gets alone, whichever requests it shared
a launch with; admission respects the device budget; launches overlap."""

import threading
import time

import numpy as np
import pytest

import oracle
import paper_2602_23967_amd as P
from paper_2602_23967_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need the MI355X"
    return T


def _mix():
    qs = [I.mpc(300 + i) for i in range(24)] + [I.mpc(400, infeasible=True)]
    qs += [I.random_small(7, n=300), I.random_small(8), I.tiny_lp(5), I.tiny_lp(6),
           I.contradictory_rows(3), I.portfolio(2, n_assets=20000, k_factors=100)]
    rng = np.random.default_rng(5)
    return [qs[i] for i in rng.permutation(len(qs))]


def _submit_poisson(srv, qs, mean_gap_s, seed=0):
    rng = np.random.default_rng(seed)
    ids = [None] * len(qs)

    def run():
        for i, q in enumerate(qs):
            time.sleep(rng.exponential(mean_gap_s))
            ids[i] = srv.submit(q)

    t = threading.Thread(target=run)
    t.start()
    t.join()
    return ids


def _general(q):
    import scipy.sparse as sp
    if q.Q is None:
        return False
    r, c = sp.csr_matrix(q.Q).nonzero()
    return bool(np.any(r != c))


def _alone(q, params, route):
    if route == 0:
        with P.BatchSolver([q]) as bs:
            # the server's general lanes use the shape for inner solves
            if _general(q):
                bs.set_schedule(P.qp_batch_default_shape(True), -1)
            bs.solve(params)
            return bs.result(0)
    with P.Solver(q) as s:
        return s.solve(params)


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_serve_result_same_alone_and_in_the_mix(torch, precision):
    qs = _mix()
    params = P.qp_params_default(precision=precision)
    with P.Server(params, batch_lanes=3, single_workers=2, batch_linger_us=300.0) as srv:
        ids = _submit_poisson(srv, qs, 2e-4)
        out = []
        for rid in ids:
            st = srv.wait(rid, 120.0)
            assert st > 0
            out.append(srv.result(rid))
    routes = set()
    for q, (g, t) in zip(qs, out):
        routes.add(t["route"])
        assert t["submitted"] <= t["started"] <= t["finished"]
        a = _alone(q, params, t["route"])
        assert g.status == a.status, q.name
        assert g.info["iterations"] == a.info["iterations"], q.name
        assert np.array_equal(g.x, a.x) and np.array_equal(g.y, a.y), q.name
        if g.status == P.OPTIMAL:
            k = oracle.kkt(q, g.x, g.y)
            assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6, q.name
    assert routes == {0, 1}


def test_serve_statuses_match_oracle(torch):
    qs = [I.mpc(500), I.mpc(501, infeasible=True), I.contradictory_rows(4), I.unbounded_qp(2),
          I.random_small(9, n=200)]
    with P.Server() as srv:
        ids = [srv.submit(q) for q in qs]
        res = []
        for rid in ids:
            srv.wait(rid, 120.0)
            res.append(srv.result(rid)[0])
    for q, g in zip(qs, res):
        o = oracle.solve(q, max_iter=100000)
        assert g.status == o.status, (q.name, g.status_name, o.status_name)


def test_serve_budget_admission_and_overlap(torch):
    """A budget that holds only a few MPC instances at once: every request
    still completes, no launch exceeds what the budget admits, and launches
    of different lanes run at the same time."""
    qs = [I.mpc(600 + i) for i in range(60)]
    # above any one instance's device bytes: the budget admits 12 to 17 at once
    one = max(16 * 2 * q.nnz_A + 8 * 30 * (q.n + q.m) for q in qs)
    with P.Server(batch_lanes=4, single_workers=0, device_budget=12 * one, max_batch=4,
                  batch_linger_us=0.0) as srv:
        ids = [srv.submit(q) for q in qs]
        times = []
        for rid in ids:
            assert srv.wait(rid, 120.0) == P.OPTIMAL
            times.append(srv.result(rid)[1])
    assert all(t["batch_size"] <= 4 for t in times)
    spans = sorted({(t["started"], t["finished"]) for t in times})
    overlap = any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert overlap, spans


def test_serve_errors(torch):
    q = I.mpc(700)
    with P.Server(batch_linger_us=2e6, single_workers=0) as srv:
        rid = srv.submit(q)
        with pytest.raises(P.QPError) as e:       # still waiting in the queue
            P.qp_server_result(srv.h, rid, q.n, q.m)
        assert e.value.code == P.ERR_STATE
        assert srv.wait(rid, 0.0) == P.NOT_SOLVED
        assert srv.wait(rid, 60.0) == P.OPTIMAL
        srv.result(rid)
        with pytest.raises(P.QPError) as e:
            srv.wait(rid, 0.0)                    # released
        assert e.value.code == P.ERR_INVALID_ARG
        with pytest.raises(P.QPError) as e:
            P.qp_server_submit(srv.h, q.n, q.m, q.Q, q.A, q.c, q.b, b"X" * q.m, q.lb, q.ub)
        assert e.value.code == P.ERR_INVALID_ARG


def test_serve_with_a_chosen_batch_schedule(torch):
    """A server configured with a non-default launch shape and index-order
    queue gives each batched request the result that shape gives it alone."""
    qs = [I.mpc(600 + i) for i in range(12)]
    params = P.qp_params_default(precision=P.PRECISION_MIXED)
    shape = P.qp_batch_num_shapes() - 1
    with P.Server(params, batch_lanes=2, single_workers=1, batch_shape=shape, batch_order=0) as srv:
        ids = [srv.submit(q) for q in qs]
        out = []
        for rid in ids:
            assert srv.wait(rid, 120.0) > 0
            out.append(srv.result(rid))
    for q, (g, t) in zip(qs, out):
        assert t["route"] == 0
        with P.BatchSolver([q]) as bs:
            bs.set_schedule(shape, 0)
            bs.solve(params)
            a = bs.result(0)
        assert g.status == a.status == P.OPTIMAL, q.name
        assert np.array_equal(g.x, a.x) and np.array_equal(g.y, a.y), q.name


def test_serve_single_path_worker_classes(torch):
    """No batched lanes: every request runs on the single-problem path, the
    diagonal-Q ones on the reserved worker, the others on the general one
    (or on the reserved one only when no general worker exists)."""
    qs = [I.portfolio(5, n_assets=10000, k_factors=50), I.random_small(11), I.tiny_lp(8),
          I.random_small(12, n=300), I.mpc(700)]
    params = P.qp_params_default()
    for cfg in ({"single_workers": 2, "diag_workers": 1}, {"single_workers": 1, "diag_workers": 1}):
        with P.Server(params, batch_lanes=0, general_lanes=0, **cfg) as srv:
            ids = [srv.submit(q) for q in qs]
            out = []
            for rid in ids:
                assert srv.wait(rid, 120.0) > 0, cfg
                out.append(srv.result(rid))
        for q, (g, t) in zip(qs, out):
            assert t["route"] == 1, (cfg, q.name)
            a = _alone(q, params, 1)
            assert g.status == a.status, (cfg, q.name)
            assert np.array_equal(g.x, a.x) and np.array_equal(g.y, a.y), (cfg, q.name)
