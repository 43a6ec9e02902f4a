"""Degenerate problems on the HIP path, against the oracle and exact
answers: one variable with no rows, one variable with one row, an empty row
(always satisfied, or infeasible on its own), a fixed variable, a variable
with no quadratic term, and an LP whose every feasible point is optimal.
Each runs through the single-problem path and, all together, through one
batched launch."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2602_23967_amd as P
from paper_2602_23967_amd import instances as I
from bruteforce import qp_enum, lc_uc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need the MI355X"
    T.cuda.init()
    return T


def _qp(name, Q, A, c, b, sense, lb, ub):
    Q = None if Q is None else sp.csr_matrix(np.asarray(Q, dtype=float))
    A = sp.csr_matrix(np.asarray(A, dtype=float).reshape(len(sense), len(c)))
    return I.QP(n=len(c), m=len(sense), Q=Q, A=A, c=np.asarray(c, dtype=float),
                b=np.asarray(b, dtype=float), sense=sense, lb=np.asarray(lb, dtype=float),
                ub=np.asarray(ub, dtype=float), name=name)


def _cases():
    return {
        # min x^2 - 3x on [0, 1]: the unconstrained minimiser 1.5 clipped to 1
        "one_var_no_rows": _qp("one_var_no_rows", [[2.0]], np.zeros((0, 1)), [-3.0], [], b"",
                               [0.0], [1.0]),
        # min x^2/2 + x with 2x >= 1 on [-5, 5]: the row is active, x = 0.5
        "one_var_one_row": _qp("one_var_one_row", [[1.0]], [[2.0]], [1.0], [1.0], b"G", [-5.0], [5.0]),
        # x0 + x1 + x2 = 1; an empty row with 0 >= -1; x0 - x2 <= 0.2;
        # x1 fixed at 0.3; no quadratic term on x1
        "empty_row_fixed_var": _qp("empty_row_fixed_var", np.diag([1.0, 0.0, 2.0]),
                                   [[1, 1, 1], [0, 0, 0], [1, 0, -1]], [0.1, 0.3, -0.2],
                                   [1.0, -1.0, 0.2], b"EGL", [0.0, 0.3, -1.0], [1.0, 0.3, 1.0]),
        # an LP whose objective is zero: every feasible point is optimal
        "zero_objective_lp": _qp("zero_objective_lp", None, [[1, 2, 0, -1], [0, 1, 1, 1]], np.zeros(4),
                                 [1.0, 0.5], b"EG", [-1.0, -1.0, 0.0, 0.0], [2.0, 2.0, 1.0, 1.0]),
    }


def _exact(q):
    Q = np.zeros((q.n, q.n)) if q.Q is None else q.Q.toarray()
    lc, uc = lc_uc(q.b, q.sense)
    return qp_enum(Q, q.c, q.A.toarray(), lc, uc, q.lb, q.ub)


def _check_optimal(q, r, what):
    assert r.status == P.OPTIMAL, (what, q.name, r.status)
    k = oracle.kkt(q, r.x, r.y)
    assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6, (what, q.name, k)
    assert np.all(r.x >= q.lb) and np.all(r.x <= q.ub)
    _, f = _exact(q)
    err = abs(r.info["primal_obj"] - f) / (1 + abs(f))
    print(f"{what} {q.name}: objective {r.info['primal_obj']!r} vs exact {f!r} ({err:.1e})", flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("name", list(_cases()))
@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_degenerate_single(torch, name, precision):
    q = _cases()[name]
    with P.Solver(q) as s:
        g = s.solve(precision=precision)
    o = oracle.solve(q)
    assert o.status == P.OPTIMAL
    _check_optimal(q, g, "gpu")
    if name != "zero_objective_lp":              # unique minimiser
        x, _ = _exact(q)
        assert np.abs(g.x - x).max() <= 1e-5, (g.x, x)
        assert np.abs(g.x - o.x).max() <= 1e-5, (g.x, o.x)


def test_empty_row_infeasible(torch):
    """0 >= 1 in an empty row: primal infeasible, the certificate on that row."""
    q = _qp("empty_row_infeasible", np.eye(2), [[1, 1], [0, 0]], [0.0, 0.0], [1.0, 1.0], b"EG",
            [-1.0, -1.0], [1.0, 1.0])
    o = oracle.solve(q)
    with P.Solver(q) as s:
        g = s.solve()
    assert g.status == o.status == P.PRIMAL_INFEASIBLE
    assert abs(g.y[1]) > 0.0 and abs(g.y[1]) >= abs(g.y[0])


def test_degenerate_batch(torch):
    """The same problems as instances of one batched launch."""
    qs = list(_cases().values())
    with P.BatchSolver(qs) as b:
        st, _ = b.solve()
        for i, q in enumerate(qs):
            r = b.result(i)
            assert st[i] == r.status
            _check_optimal(q, r, "batch")
