"""Pins of the oracle's primal-subproblem solvers (Section 2.2): the
subproblem is strictly convex, so its minimiser is unique and exact references
exist: a dense linear solve when unboxed, 3^n enumeration when boxed."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2602_23967_amd import instances as I
from bruteforce import box_qp_enum


def _kkt_signs(H, r, x, l, u, tol):
    g = H @ x - r
    free = (x > l) & (x < u)
    assert np.all(np.abs(g[free]) <= tol)
    atl = (x <= l) & (l < u)
    atu = (x >= u) & (l < u)
    assert np.all(g[atl] >= -tol)
    assert np.all(g[atu] <= tol)
    assert np.all(x >= l) and np.all(x <= u)


@pytest.mark.parametrize("solver", [oracle.INNER_MPRGP, oracle.INNER_BB])
def test_unboxed_matches_dense_solve(solver):
    q = I.random_small(0)
    n = q.n
    tau = 0.37
    rng = np.random.default_rng(5)
    rhs = rng.normal(size=n)
    H = q.Q.toarray() + np.eye(n) / tau
    xs = np.linalg.solve(H, rhs)
    x, it, res = oracle.subproblem(q.Q, np.full(n, -np.inf), np.full(n, np.inf), tau, rhs,
                                   np.zeros(n), 1e-11, max_inner=20000, solver=solver)
    assert res <= 1e-11
    assert np.abs(x - xs).max() <= 1e-9 * (1 + np.abs(xs).max())


@pytest.mark.parametrize("inst", range(6))
@pytest.mark.parametrize("solver", [oracle.INNER_MPRGP, oracle.INNER_BB])
def test_boxed_matches_enumeration(inst, solver):
    rng = np.random.default_rng(100 + inst)
    n = 7
    B = rng.normal(size=(n, n))
    Qd = B.T @ B * 0.3
    tau = rng.uniform(0.2, 2.0)
    H = Qd + np.eye(n) / tau
    r = rng.normal(size=n) * 4
    l = -np.ones(n) * rng.uniform(0.2, 1.0, n)
    u = np.ones(n) * rng.uniform(0.2, 1.0, n)
    if inst % 2:
        l[0] = -np.inf          # one-sided and free coordinates
        u[1] = np.inf
        l[2], u[2] = -np.inf, np.inf
    if inst == 4:
        l[3] = u[3] = 0.25      # a fixed variable
    xs = box_qp_enum(H, r, l, u)
    x, it, res = oracle.subproblem(sp.csr_matrix(Qd), l, u, tau, r, np.zeros(n), 1e-12,
                                   max_inner=20000, solver=solver)
    assert res <= 1e-12
    assert np.abs(x - xs).max() <= 1e-9


def test_closed_form_diagonal_kkt():
    rng = np.random.default_rng(3)
    n = 50
    d = rng.uniform(0.0, 2.0, n)
    Qd = sp.diags(d).tocsr()
    tau = 0.8
    r = rng.normal(size=n) * 3
    l = np.where(rng.uniform(size=n) < 0.2, -np.inf, -1.0)
    u = np.where(rng.uniform(size=n) < 0.2, np.inf, 1.0)
    x, it, res = oracle.subproblem(Qd, l, u, tau, r, np.zeros(n), 0.0,
                                   solver=oracle.INNER_CLOSED)
    assert it == 0
    _kkt_signs(np.diag(d) + np.eye(n) / tau, r, x, l, u, 1e-13)
    with pytest.raises(ValueError):
        oracle.subproblem(I.random_small(0).Q, np.full(1000, -1.0), np.full(1000, 1.0), tau,
                          np.zeros(1000), np.zeros(1000), 0.0, solver=oracle.INNER_CLOSED)


def test_mprgp_and_bb_agree_medium_boxed():
    """Both solvers reach the unique minimiser of a 1000-variable boxed
    subproblem with many active bounds; the sign conditions hold."""
    q = I.random_small(1)
    n = q.n
    tau = 0.15
    rng = np.random.default_rng(9)
    r = rng.normal(size=n) * 20
    H = q.Q.toarray() + np.eye(n) / tau
    l, u = q.lb, q.ub
    x1, it1, r1 = oracle.subproblem(q.Q, l, u, tau, r, np.zeros(n), 1e-11, 20000,
                                    oracle.INNER_MPRGP)
    x2, it2, r2 = oracle.subproblem(q.Q, l, u, tau, r, np.zeros(n), 1e-11, 20000,
                                    oracle.INNER_BB)
    active = np.mean((x1 <= l) | (x1 >= u))
    assert active > 0.3
    assert np.abs(x1 - x2).max() <= 1e-9
    _kkt_signs(H, r, x1, l, u, 1e-10)


def test_mixed_bounds_subproblem():
    q = I.mixed_bounds(0)
    n = q.n
    tau = 0.5
    rng = np.random.default_rng(2)
    r = rng.normal(size=n) * 5
    x, it, res = oracle.subproblem(q.Q, q.lb, q.ub, tau, r, np.zeros(n), 1e-11, 20000,
                                   oracle.INNER_MPRGP)
    H = q.Q.toarray() + np.eye(n) / tau
    _kkt_signs(H, r, x, q.lb, q.ub, 1e-10)
    fixed = q.lb == q.ub
    assert np.all(x[fixed] == q.lb[fixed])


def test_warm_start_at_solution_takes_no_iteration():
    q = I.random_small(0)
    n = q.n
    r = np.random.default_rng(4).normal(size=n)
    x, it, res = oracle.subproblem(q.Q, q.lb, q.ub, 0.3, r, np.zeros(n), 1e-10, 20000)
    x2, it2, res2 = oracle.subproblem(q.Q, q.lb, q.ub, 0.3, r, x, 1e-8, 20000)
    assert it > 0 and it2 == 0


def test_unboxed_cg_finite_termination():
    """With no active bound MPRGP is conjugate gradients, which solves an
    n x n SPD system in at most n steps in exact arithmetic; a lost
    conjugacy (wrong coefficient) shows up as many more steps."""
    rng = np.random.default_rng(11)
    n = 12
    B = rng.normal(size=(n, n))
    Qd = B.T @ B / n + 0.05 * np.eye(n)
    r = rng.normal(size=n)
    inf = np.full(n, np.inf)
    x, it, res = oracle.subproblem(sp.csr_matrix(Qd), -inf, inf, 10.0, r, np.zeros(n), 1e-10,
                                   max_inner=1000, solver=oracle.INNER_MPRGP)
    assert res <= 1e-10
    assert it <= n + 2
