"""Pins of the oracle's full solve and KKT evaluation against exact
references: dense KKT solves, active-set enumeration, HiGHS on LPs, and
constructed infeasible / unbounded instances with known certificates
(Sections 2, 4 and 5)."""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle
from paper_2602_23967_amd import instances as I
from bruteforce import lc_uc, qp_enum


def _dense(q):
    Q = np.zeros((q.n, q.n)) if q.Q is None else q.Q.toarray()
    return Q, q.A.toarray()


def _box(l, u):
    return [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
            for a, b in zip(l, u)]


# ---- KKT residual definitions (Section 4) ------------------------------------

@pytest.mark.parametrize("inst", range(3))
def test_kkt_zero_at_exact_equality_solution(inst):
    """At the exact solution of an equality-only unboxed QP (a dense linear
    KKT solve with r = Qx + c + A'y = 0) all three residuals vanish and the
    primal and dual objectives coincide (no dropped term or sign error can
    survive this)."""
    q = I.equality_qp(inst)
    Q, A = _dense(q)
    K = np.block([[Q, A.T], [A, np.zeros((q.m, q.m))]])
    sol = np.linalg.solve(K, np.concatenate([-q.c, q.b]))
    x, y = sol[: q.n], sol[q.n:]
    k = oracle.kkt(q, x, y)
    assert k["r_primal"] < 1e-13 and k["r_dual"] < 1e-12 and k["r_gap"] < 1e-12
    assert k["pobj"] == pytest.approx(0.5 * x @ Q @ x + q.c @ x, rel=1e-13)
    assert k["dobj"] == pytest.approx(k["pobj"], rel=1e-11)


@pytest.mark.parametrize("inst", range(4))
def test_kkt_gap_zero_at_boxed_optimum(inst):
    """Boxed tiny QP: the enumerated optimum with multipliers recovered from
    the active rows gives zero gap; any feasible x has r_primal = 0 and any
    point with a row off by delta has r_primal = delta / (1 + max|b|)."""
    q = I.tiny(inst, n=5, m=3)
    Q, A = _dense(q)
    lc, uc = lc_uc(q.b, q.sense)
    xs, fs = qp_enum(Q, q.c, A, lc, uc, q.lb, q.ub)
    # dual: solve min over (x, y) feasible of the oracle objective at tight tol
    r = oracle.solve(q, tol=1e-10, eps_min=1e-13, max_iter=200000)
    assert r.status == oracle.OPTIMAL
    k = oracle.kkt(q, xs, r.y)
    assert k["r_primal"] < 1e-9
    assert k["r_gap"] < 1e-8
    assert k["pobj"] == pytest.approx(fs, rel=1e-12, abs=1e-12)
    # primal residual is exactly the scaled worst row violation
    x2 = xs.copy()
    x2[0] += 0.3
    viol = A @ x2 - np.clip(A @ x2, lc, uc)
    bscale = 1 + max(np.abs(lc[np.isfinite(lc)]).max(initial=0), np.abs(uc[np.isfinite(uc)]).max(initial=0))
    assert oracle.kkt(q, x2, r.y)["r_primal"] == pytest.approx(np.abs(viol).max() / bscale, rel=1e-12)


def test_weak_duality_of_dual_objective():
    """For a feasible x and any y in Y the dual objective of eq. dualQP never
    exceeds the primal objective of any feasible point (weak duality)."""
    q = I.tiny(7, n=5, m=3)
    Q, A = _dense(q)
    lc, uc = lc_uc(q.b, q.sense)
    x0 = q.meta["x0"]
    rng = np.random.default_rng(0)
    for _ in range(50):
        y = rng.normal(size=q.m) * 3
        y = np.where(np.isfinite(lc) & ~np.isfinite(uc), np.minimum(y, 0), y)   # R- for '>='
        y = np.where(~np.isfinite(lc) & np.isfinite(uc), np.maximum(y, 0), y)   # R+ for '<='
        xr = rng.uniform(-1, 1, q.n)
        k = oracle.kkt(q, xr, y)
        assert k["dobj"] <= 0.5 * x0 @ Q @ x0 + q.c @ x0 + 1e-10


# ---- full solves against exact references --------------------------------------

@pytest.mark.parametrize("inst", range(3))
def test_equality_qp_matches_dense_kkt(inst):
    q = I.equality_qp(inst)
    Q, A = _dense(q)
    K = np.block([[Q, A.T], [A, np.zeros((q.m, q.m))]])
    sol = np.linalg.solve(K, np.concatenate([-q.c, q.b]))
    xs, ys = sol[: q.n], sol[q.n:]
    r = oracle.solve(q, tol=1e-9)
    assert r.status == oracle.OPTIMAL
    assert np.abs(r.x - xs).max() <= 1e-6 * (1 + np.abs(xs).max())
    assert np.abs(r.y - ys).max() <= 1e-5 * (1 + np.abs(ys).max())


@pytest.mark.parametrize("inst", range(5))
def test_tiny_boxed_qp_matches_enumeration(inst):
    q = I.tiny(inst, n=5, m=3)
    Q, A = _dense(q)
    lc, uc = lc_uc(q.b, q.sense)
    xs, fs = qp_enum(Q, q.c, A, lc, uc, q.lb, q.ub)
    r = oracle.solve(q, tol=1e-9, max_iter=200000)
    assert r.status == oracle.OPTIMAL
    assert r.info["primal_obj"] == pytest.approx(fs, rel=1e-7, abs=1e-7)
    assert np.abs(r.x - xs).max() <= 1e-5


def test_tiny_mixed_bounds_matches_enumeration():
    """free, one-sided and fixed variables (enumeration handles each kind)."""
    q = I.tiny(11, n=5, m=3, boxed=False)
    q.lb = np.array([-1.0, -np.inf, 0.2, -np.inf, -0.5])
    q.ub = np.array([1.0, 0.5, 0.2, np.inf, np.inf])
    Q, A = _dense(q)
    lc, uc = lc_uc(q.b, q.sense)
    xs, fs = qp_enum(Q, q.c, A, lc, uc, q.lb, q.ub)
    r = oracle.solve(q, tol=1e-9, max_iter=200000)
    assert r.status == oracle.OPTIMAL
    assert r.info["primal_obj"] == pytest.approx(fs, rel=1e-7, abs=1e-7)
    assert np.abs(r.x - xs).max() <= 1e-5
    assert r.x[2] == 0.2


@pytest.mark.parametrize("inst", range(4))
def test_lp_matches_highs(inst):
    q = I.tiny_lp(inst)
    A = q.A.toarray()
    lc, uc = lc_uc(q.b, q.sense)
    eq = lc == uc
    A_ub = np.vstack([A[~eq & np.isfinite(uc)], -A[~eq & np.isfinite(lc)]])
    b_ub = np.concatenate([uc[~eq & np.isfinite(uc)], -lc[~eq & np.isfinite(lc)]])
    ref = linprog(q.c, A_ub=A_ub, b_ub=b_ub, A_eq=A[eq], b_eq=lc[eq],
                  bounds=_box(q.lb, q.ub), method="highs")
    assert ref.status == 0
    r = oracle.solve(q, tol=1e-8, max_iter=400000)
    assert r.status == oracle.OPTIMAL
    assert r.info["primal_obj"] == pytest.approx(ref.fun, rel=1e-6, abs=1e-6)


def test_random_small_workload_is_optimal():
    """n = 1000 workload instance: OPTIMAL at 1e-6, and the returned point
    passes an independent NumPy check of primal feasibility and of the
    gap's definition (Section 4)."""
    q = I.random_small(0)
    r = oracle.solve(q)
    assert r.status == oracle.OPTIMAL
    assert max(r.info["r_primal"], r.info["r_dual"], r.info["r_gap"]) <= 1e-6
    Q, A = _dense(q)
    lc, uc = lc_uc(q.b, q.sense)
    ax = A @ r.x
    assert np.abs(ax - np.clip(ax, lc, uc)).max() <= 1e-6 * (1 + np.abs(q.b).max())
    assert np.all(r.x >= q.lb) and np.all(r.x <= q.ub)
    # y in Y: '=' rows free, '>=' rows nonpositive
    assert np.all(r.y[q.m // 2:] <= 0)
    # tighter solve changes the objective by less than the tolerance predicts
    r2 = oracle.solve(q, tol=1e-9)
    assert r2.status == oracle.OPTIMAL
    assert r.info["primal_obj"] == pytest.approx(r2.info["primal_obj"], rel=1e-5)


# ---- infeasibility (Section 5) -----------------------------------------------

def _separation(q, ray):
    """inf_{x in X} ray'Ax and sup_{s in S} ray's, each by an LP."""
    A = q.A.toarray()
    lc, uc = lc_uc(q.b, q.sense)
    w = A.T @ ray
    lo = linprog(w, bounds=_box(q.lb, q.ub), method="highs")
    hi = linprog(-ray, bounds=_box(lc, uc), method="highs")
    return lo.fun, -hi.fun


@pytest.mark.parametrize("make", [lambda: I.contradictory_rows(0), lambda: I.contradictory_rows(1),
                                  lambda: I.box_infeasible_rows(0),
                                  lambda: I.random_small(0, infeasible=True)])
def test_primal_infeasible_certificate(make):
    q = make()
    A = q.A.toarray()
    lc, uc = lc_uc(q.b, q.sense)
    eq = lc == uc
    A_ub = np.vstack([A[~eq & np.isfinite(uc)], -A[~eq & np.isfinite(lc)]])
    b_ub = np.concatenate([uc[~eq & np.isfinite(uc)], -lc[~eq & np.isfinite(lc)]])
    ph1 = linprog(np.zeros(q.n), A_ub=A_ub if len(b_ub) else None, b_ub=b_ub if len(b_ub) else None,
                  A_eq=A[eq], b_eq=lc[eq], bounds=_box(q.lb, q.ub), method="highs")
    assert ph1.status == 2            # HiGHS confirms infeasibility
    r = oracle.solve(q, max_iter=20000)
    assert r.status == oracle.PRIMAL_INFEASIBLE
    ray = r.y
    assert np.abs(ray).max() == pytest.approx(1.0)
    inf_x, sup_s = _separation(q, ray)
    assert inf_x > sup_s + 1e-9        # strict separation proves A X and S are disjoint


def test_unbounded_certificate():
    q = I.unbounded_qp(0)
    r = oracle.solve(q, max_iter=20000)
    assert r.status == oracle.DUAL_INFEASIBLE
    d = r.x
    Q, A = _dense(q)
    # theorem conditions: d in Recc X, A d in Recc S (= {0} for '=' rows), c'd < 0, Q d = 0
    assert np.abs(d).max() == pytest.approx(1.0)
    fin = np.isfinite(q.lb) & np.isfinite(q.ub)
    assert np.all(d[fin] == 0) and np.all(d[~np.isfinite(q.lb)] <= 0)
    assert np.abs(A @ d).max() <= 1e-8 and np.abs(Q @ d).max() <= 1e-8
    assert q.c @ d < 0
    x0 = q.meta.get("x0", None)
    x0 = np.clip(np.zeros(q.n), q.lb, q.ub) if x0 is None else x0
    f = lambda x: 0.5 * x @ Q @ x + q.c @ x
    assert f(x0 + 1e6 * d) < f(x0) - 1e5


def test_large_sparse_infeasible_variant_small():
    q = I.large_sparse(0, n=4000, infeasible=True)
    r = oracle.solve(q, max_iter=20000)
    assert r.status == oracle.PRIMAL_INFEASIBLE
    r1, r2 = q.meta["rows"]
    big = np.argsort(-np.abs(r.y))[:2]
    assert set(big) == {r1, r2}
    assert r.y[r1] * r.y[r2] < 0


# ---- limits and edge cases ---------------------------------------------------

def test_iteration_limits():
    q = I.random_small(0)
    r0 = oracle.solve(q, max_iter=0)
    assert r0.status == oracle.ITERATION_LIMIT and r0.info["iterations"] == 0
    assert np.all(r0.x == 0) and np.all(r0.y == 0)      # proj_X(0) with 0 in the box
    r1 = oracle.solve(q, max_iter=1)
    assert r1.status == oracle.ITERATION_LIMIT and r1.info["iterations"] == 1


def test_no_rows():
    """m = 0: the problem is a box-constrained QP; the solution is the
    subproblem minimiser with tau -> infinity (checked by enumeration)."""
    q = I.tiny(21, n=5, m=1)
    q.A = q.A[:0]
    q.b = q.b[:0]
    q.sense = b""
    q.m = 0
    Q, _ = _dense(q)
    xs, fs = qp_enum(Q, q.c, np.zeros((0, q.n)), np.zeros(0), np.zeros(0), q.lb, q.ub)
    r = oracle.solve(q, tol=1e-10)
    assert r.status == oracle.OPTIMAL
    assert np.abs(r.x - xs).max() <= 1e-6


def test_adaptive_inner_tolerance_saves_inner_iterations():
    """The idea of the ablation in Section 6.3: the adaptive rule reaches the
    same status with fewer inner iterations than a fixed 1e-9 tolerance."""
    q = I.random_small(1)
    a = oracle.solve(q)
    f = oracle.solve(q, eps_inner_fixed=1e-9)
    assert a.status == f.status == oracle.OPTIMAL
    assert a.info["inner_iterations"] < f.info["inner_iterations"]


def test_plain_pdhg_reaches_same_solution():
    q = I.random_small(2)
    a = oracle.solve(q, tol=1e-8)
    b = oracle.solve(q, tol=1e-8, use_halpern=0)
    assert a.status == b.status == oracle.OPTIMAL
    assert np.abs(a.x - b.x).max() <= 1e-4
    assert a.info["primal_obj"] == pytest.approx(b.info["primal_obj"], rel=1e-7)


def test_primal_residual_scale_uses_both_row_bounds():
    """r_primal divides by 1 + max(||l_c||_inf, ||u_c||_inf) over finite
    entries (Section 4): with '<=' rows only, l_c is all -inf and the scale
    comes from u_c alone."""
    q = I.tiny(31, n=4, m=2, senses="L")
    q.b = np.array([50.0, -3.0])
    A = q.A.toarray()
    x = np.linalg.lstsq(A, q.b + np.array([2.0, 0.0]), rcond=None)[0]   # row 0 off by 2
    k = oracle.kkt(q, x, np.zeros(2))
    viol = max((A @ x - q.b).max(), 0.0)
    assert k["r_primal"] == pytest.approx(viol / 51.0, rel=1e-10)


def test_factored_portfolio_equals_factor_variable_form():
    """Eliminating f = F w turns the factor-variable portfolio into the
    factored one: the oracle reaches the same w and objective on both."""
    import paper_2602_23967_amd.instances as I
    qf = I.portfolio_factored(7, n_assets=400, k_factors=8)
    qv = I.portfolio(7, n_assets=400, k_factors=8)
    e = qf.explicit()
    Fd = qf.R.toarray()
    assert np.allclose(e.Q.toarray(), qf.Q.toarray() + Fd.T @ Fd, rtol=0, atol=1e-15)
    a = oracle.solve(e, tol=1e-9, max_iter=400000)
    b = oracle.solve(qv, tol=1e-9, max_iter=400000)
    assert a.status == b.status == oracle.OPTIMAL
    assert a.info["primal_obj"] == pytest.approx(b.info["primal_obj"], rel=1e-7, abs=1e-9)
    assert np.abs(a.x - b.x[:400]).max() <= 1e-5


def _hand_case_qp(c):
    import scipy.sparse as sp
    return I.QP(n=3, m=2, Q=sp.csr_matrix(np.diag([4.0, 3.0, 0.0])),
                A=sp.csr_matrix(np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 1.0]])),
                c=np.array(c, dtype=np.float64), b=np.array([2.0, 1.0]), sense=b"EG",
                lb=np.array([-1.0, -np.inf, -np.inf]), ub=np.array([np.inf, 2.0, np.inf]),
                name="kkt_hand")


def _hand_cases():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "kkt_hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"])
def test_kkt_normalisations_match_hand_worked_values(case):
    """Section 4's three residuals with nonzero numerators, each denominator
    term of r_dual (||Qx||, ||A'y||, ||c||) and of r_gap (|primal objective|,
    |x'Qx/2 + p(-rhat) + p(y)|, either sign) made to dominate in turn, on a
    3-variable problem with a lower-bounded, an upper-bounded and a free
    variable, against exact rationals worked by hand (the derivation is in
    the fixture).  A 2-norm in place of an infinity norm, a dropped term, a
    missing absolute value or the gap taken at r instead of proj_R(r) fails
    at least one case."""
    from fractions import Fraction
    q = _hand_case_qp(case["c"])
    k = oracle.kkt(q, np.array([1.0, 1.0, 0.5]), np.array(case["y"], dtype=np.float64))
    for key in ("r_primal", "r_dual", "r_gap", "pobj", "dobj", "natural", "pviol"):
        want = float(Fraction(case[key]))
        assert k[key] == pytest.approx(want, rel=1e-14, abs=1e-300), key


# ---- Halpern anchoring (Section 3.1) -----------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_halpern_limit_is_projection_of_anchor(seed):
    """Without restarts, Halpern iterates of a nonexpansive map converge to
    the point of its fixed-point set nearest the anchor, in the norm that
    makes the map nonexpansive (Wittmann's theorem).  For an LP with c = 0
    whose feasible set has a point inside the box, every feasible x is
    optimal and y* = 0 is the only dual solution; with the anchor's y at 0
    that norm reduces to the Euclidean one on x, so the limit is the
    projection of the anchor x0 = proj_box(0) onto {Ax = b, l <= x <= u},
    found here by active-set enumeration.  Plain PDHG (no anchor) reaches
    another optimal x on most of these instances, and an anchor other than
    the starting point moves the limit."""
    rng = np.random.default_rng(seed)
    n, m = 5, 2
    A = rng.normal(size=(m, n))
    lb = rng.uniform(-1.0, 0.5, n)
    ub = lb + rng.uniform(0.3, 2.0, n)
    b = A @ rng.uniform(lb, ub)
    q = I.QP(n=n, m=m, Q=None, A=sp.csr_matrix(A), c=np.zeros(n), b=b, sense=b"EE", lb=lb, ub=ub,
             name=f"halpern_limit_{seed}")
    x0 = np.clip(0.0, lb, ub)
    p, _ = qp_enum(np.eye(n), -x0, A, b, b, lb, ub)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)           # five variables: threads only add overhead
    try:
        r = oracle.solve(q, max_iter=100000, check_every=10**12, tol=0.0)
        plain = oracle.solve(q, max_iter=100000, check_every=10**12, tol=0.0, use_halpern=0)
    finally:
        oracle.set_num_threads(threads)
    assert r.status == oracle.ITERATION_LIMIT
    err = np.abs(r.x - p).max()
    assert err <= 5e-5, err
    assert np.abs(r.y).max() <= 5e-5
    assert np.abs(A @ plain.x - b).max() <= 1e-9
    if seed in (0, 1, 2, 3, 6):
        assert np.abs(plain.x - p).max() >= 1e-2
    # the projection of 0 itself: where an anchor at the origin would lead
    p_origin, _ = qp_enum(np.eye(n), np.zeros(n), A, b, b, lb, ub)
    if seed in (0, 1, 3, 4, 5, 6):
        assert np.abs(p_origin - p).max() >= 1e-2
