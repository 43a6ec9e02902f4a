"""The allocation-free batched entry point (qp_batch_solve_static) against
the allocating one (qp_batch_create + qp_batch_solve + qp_batch_result) on
the same instances: same statuses and bitwise-equal x, y and outcomes, on two
calls in a row, the second smaller (the static workspace then still holds
the first call's larger contents); a batch too large for the workspace is
refused with a clear error and the next call still works."""

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


def _first_mix():
    qs = [I.mpc(i) for i in range(24)]
    qs += [I.mpc(200, infeasible=True), I.tiny_lp(5)]
    qs += [I.random_small(3, n=300), I.mixed_bounds(2), I.contradictory_rows(2), I.unbounded_qp(2)]
    return qs


def _second_mix():
    # fewer and different instances, so stale workspace contents would show
    return [I.mpc(300 + i) for i in range(6)] + [I.random_small(5, n=200), I.tiny(7, n=6, m=3)]


def _static(qs, params=None, stream=None):
    big, vo, ro = I.pack(qs)
    print(f"static call: {len(qs)} instances, n={big.n} m={big.m}", flush=True)
    return P.qp_batch_solve_static(len(qs), vo, ro, big.Q, big.A, big.c, big.b, big.sense, big.lb, big.ub,
                                   params=params, stream=stream)


def _allocating(qs, params=None):
    print(f"allocating path: {len(qs)} instances", flush=True)
    with P.BatchSolver(qs) as bs:
        st, _ = bs.solve(params)
        res = [bs.result(i) for i in range(len(qs))]
    return st, res


def _compare(qs, got, ref):
    opt, x, y, st, infos = got
    st_ref, res = ref
    assert opt == int(np.sum(np.asarray(st_ref) == P.OPTIMAL))
    assert list(st) == list(st_ref)
    _, vo, ro = I.pack(qs)
    for i, (q, r) in enumerate(zip(qs, res)):
        assert st[i] == r.status, q.name
        assert np.array_equal(x[vo[i]:vo[i + 1]], r.x), q.name
        assert np.array_equal(y[ro[i]:ro[i + 1]], r.y), q.name
        for k in ("iterations", "inner_iterations", "restarts", "r_primal", "r_dual", "r_gap",
                  "primal_obj", "dual_obj"):
            assert infos[i][k] == r.info[k], (q.name, k, infos[i][k], r.info[k])


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_static_equals_allocating_two_calls(torch, precision):
    params = P.qp_params_default(precision=precision)
    first, second = _first_mix(), _second_mix()
    got1 = _static(first, params)
    _compare(first, got1, _allocating(first, params))
    got2 = _static(second, params)
    _compare(second, got2, _allocating(second, params))
    # and the oracle's statuses (the allocating path is checked against the
    # oracle instance by instance elsewhere)
    for q, s_ in zip(second, got2[3]):
        assert s_ == oracle.solve(q, max_iter=100000).status, q.name


def test_static_on_a_torch_stream(torch):
    qs = _second_mix()
    s = torch.cuda.Stream()
    got = _static(qs, stream=s.cuda_stream)
    _compare(qs, got, _allocating(qs))


def test_static_refuses_a_batch_beyond_the_workspace(torch):
    qs = [I.mpc(i, horizon=50) for i in range(260)]
    big, vo, ro = I.pack(qs)
    with pytest.raises(P.QPError) as e:
        P.qp_batch_solve_static(len(qs), vo, ro, big.Q, big.A, big.c, big.b, big.sense, big.lb, big.ub)
    assert e.value.code == P.ERR_INVALID_ARG
    assert "static workspace" in str(e.value)
    qs2 = _second_mix()
    _compare(qs2, _static(qs2), _allocating(qs2))
