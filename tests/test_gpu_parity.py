"""Parity of the HIP path with the CPU oracle, called through the C ABI.

Per-call kernels (SpMV, reductions, KKT) must match to 1e-12 relative; the
subproblem solver must reach the same unique minimiser; full solves must
return the oracle's status, a relative KKT error <= 1e-6 (evaluated by the
oracle's KKT function on the GPU's point) and the oracle's objective to
1e-6 relative.  Full-size runs of the 1e6-variable workload are checked on
sampled rows and by properties that hold at any size.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle
import paper_2602_23967_amd as P
from paper_2602_23967_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need the MI355X"
    T.cuda.init()
    return T


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    """A stored oracle result (written by tests/golden/make_oracle_golden.py)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _assert_objective(f, f_ref, what=""):
    """The acceptance bound on the objective: |f - f_ref| <= 1e-6 (1 + |f_ref|),
    f_ref from an oracle run at a tighter tolerance."""
    err = abs(f - f_ref) / (1 + abs(f_ref))
    print(f"{what} objective {f!r} vs oracle {f_ref!r}: relative error {err:.2e}", flush=True)
    assert err <= 1e-6, (what, f, f_ref)


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _box(l, u):
    return [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
            for a, b in zip(l, u)]


def _lc_uc(q):
    return oracle.bounds_from_sense(q.b, q.sense)


def _spmv_check(torch, h, op, M, x):
    xd = _dev(torch, x)
    yd = torch.zeros(M.shape[0], dtype=torch.float64, device="cuda")
    P.qp_apply(h, op, xd, yd)
    y = yd.cpu().numpy()
    ref = oracle.matvec(M, x)
    scale = abs(M) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-12 * np.maximum(scale, 1e-300) + 1e-300)


# ---- per-call kernels ----------------------------------------------------------

def test_spmv_parity_small(torch):
    q = I.random_small(0)
    h = P.qp_create_from(q)
    rng = np.random.default_rng(0)
    try:
        _spmv_check(torch, h, P.OP_Q, q.Q, rng.normal(size=q.n))
        _spmv_check(torch, h, P.OP_A, q.A, rng.normal(size=q.n))
        _spmv_check(torch, h, P.OP_AT, q.A.T.tocsr(), rng.normal(size=q.m))
    finally:
        P.qp_destroy(h)


def test_spmv_parity_ragged_rows(torch):
    """Row lengths straddling every schedule boundary: empty rows, 1..2048
    nonzeros (row blocks), 2049 and 5000 (one block's strided passes), 9000
    (segments)."""
    rng = np.random.default_rng(1)
    n = 9500
    lengths = [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 2047, 2048, 2049, 5000, 9000, 0, 7, 300, 0]
    rows, cols, vals = [], [], []
    for i, L in enumerate(lengths):
        cc = rng.choice(n, size=L, replace=False)
        rows += [i] * L
        cols += list(cc)
        vals += list(rng.normal(size=L))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(len(lengths), n))
    A.sort_indices()
    m = A.shape[0]
    h = P.qp_create(n, m, None, A, np.ones(n), np.zeros(m), b"L" * m, -np.ones(n), np.ones(n))
    try:
        for rep in range(3):
            _spmv_check(torch, h, P.OP_A, A, rng.normal(size=n))
            _spmv_check(torch, h, P.OP_AT, A.T.tocsr(), rng.normal(size=m))
            _spmv_check(torch, h, P.OP_Q, sp.csr_matrix((n, n)), rng.normal(size=n))
    finally:
        P.qp_destroy(h)


@pytest.mark.parametrize("longest", [9000, 40000])
def test_spmv_parity_wide_partitioned(torch, longest):
    """Operands wider than 262144 columns use the XCD-partitioned schedule;
    a row with more than 2048 nonzeros inside one column part (longest =
    40000) makes the library fall back to the unpartitioned schedule."""
    rng = np.random.default_rng(longest)
    n = 300_000
    lengths = [0, 1, 5, 64, 257, 2047, 2049, 5000, longest, 0, 3] + list(rng.integers(0, 40, 2000))
    rows, cols, vals = [], [], []
    for i, L in enumerate(lengths):
        cc = rng.choice(n, size=int(L), replace=False)
        rows += [i] * int(L)
        cols += list(cc)
        vals += list(rng.normal(size=int(L)))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(len(lengths), n))
    A.sort_indices()
    m = A.shape[0]
    h = P.qp_create(n, m, None, A, np.ones(n), np.zeros(m), b"L" * m, -np.ones(n), np.ones(n))
    try:
        for rep in range(2):
            _spmv_check(torch, h, P.OP_A, A, rng.normal(size=n))
            _spmv_check(torch, h, P.OP_AT, A.T.tocsr(), rng.normal(size=m))
    finally:
        P.qp_destroy(h)


@pytest.mark.parametrize("length", [0, 1, 257, 12345, 1_000_000])
def test_dot_matches_fsum(torch, length):
    q = I.tiny(0, n=4, m=2)
    h = P.qp_create_from(q)
    rng = np.random.default_rng(length)
    a = rng.normal(size=length) * np.exp(rng.normal(size=length))
    b = rng.normal(size=length)
    try:
        s = P.qp_dot(h, _dev(torch, a) if length else torch.zeros(1, dtype=torch.float64, device="cuda")[:0],
                     _dev(torch, b) if length else torch.zeros(1, dtype=torch.float64, device="cuda")[:0])
    finally:
        P.qp_destroy(h)
    ref = math.fsum(a * b)
    assert abs(s - ref) <= 1e-12 * max(np.abs(a * b).sum(), 1e-300)


def test_kkt_parity(torch):
    for q in (I.random_small(0), I.mixed_bounds(1), I.tiny_lp(0)):
        rng = np.random.default_rng(3)
        x = np.clip(rng.normal(size=q.n), q.lb, q.ub)
        y = rng.normal(size=q.m)
        lc, uc = _lc_uc(q)
        y = np.where(np.isfinite(lc) & ~np.isfinite(uc), -np.abs(y), y)
        y = np.where(~np.isfinite(lc) & np.isfinite(uc), np.abs(y), y)
        h = P.qp_create_from(q)
        try:
            g = P.qp_kkt(h, _dev(torch, x), _dev(torch, y))
        finally:
            P.qp_destroy(h)
        o = oracle.kkt(q, x, y)
        for k in o:
            assert g[k] == pytest.approx(o[k], rel=1e-11, abs=1e-13), (q.name, k)


@pytest.mark.parametrize("case", ["boxed", "unboxed", "mixed"])
def test_subproblem_parity(torch, case):
    q = I.mixed_bounds(2) if case == "mixed" else I.random_small(1)
    lv, uv = q.lb, q.ub
    if case == "unboxed":
        lv, uv = np.full(q.n, -np.inf), np.full(q.n, np.inf)
        q = I.QP(q.n, q.m, q.Q, q.A, q.c, q.b, q.sense, lv, uv)
    rng = np.random.default_rng(7)
    tau = 0.2
    rhs = rng.normal(size=q.n) * 10
    x0 = np.zeros(q.n)
    h = P.qp_create_from(q)
    try:
        xd = _dev(torch, x0)
        it, res = P.qp_subproblem(h, tau, _dev(torch, rhs), xd, 1e-10, 5000)
        xg = xd.cpu().numpy()
        nq = P.qp_norms(h)[1]
    finally:
        P.qp_destroy(h)
    xo, ito, reso = oracle.subproblem(q.Q, lv, uv, tau, rhs, x0, 1e-10, 5000,
                                      oracle.INNER_MPRGP, norm_Q=nq)
    assert res <= 1e-10 and reso <= 1e-10
    assert np.abs(xg - xo).max() <= 1e-8
    print(f"inner iterations gpu={it} oracle={ito}")


# ---- full solves ----------------------------------------------------------------

def _gpu_solve(q, **kw):
    with P.Solver(q) as s:
        return s.solve(**kw)


def _assert_kkt(q, r, tol=1e-6):
    k = oracle.kkt(q, r.x, r.y)
    assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= tol, k
    assert np.all(r.x >= q.lb) and np.all(r.x <= q.ub)
    return k


@pytest.mark.parametrize("inst", range(3))
def test_solve_random_small_matches_oracle(torch, inst):
    q = I.random_small(inst)
    g = _gpu_solve(q)
    o = oracle.solve(q)
    ref = oracle.solve(q, tol=1e-9)
    print(f"iterations gpu={g.info['iterations']}/{g.info['inner_iterations']} "
          f"oracle={o.info['iterations']}/{o.info['inner_iterations']}")
    assert g.status == o.status == P.OPTIMAL
    _assert_kkt(q, g)
    f = g.info["primal_obj"]
    fr = ref.info["primal_obj"]
    assert abs(f - fr) <= 1e-6 * (1 + abs(fr))
    assert abs(f - 0.5 * g.x @ (q.Q @ g.x) - q.c @ g.x) <= 1e-9 * (1 + abs(f))


def test_solve_is_deterministic(torch):
    q = I.random_small(0)
    with P.Solver(q) as s:
        a = s.solve()
        b = s.solve()
    assert a.info["iterations"] == b.info["iterations"]
    assert a.info["inner_iterations"] == b.info["inner_iterations"]
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)


def test_equality_qp_cg_path_matches_dense_kkt(torch):
    q = I.equality_qp(0)
    Q, A = q.Q.toarray(), q.A.toarray()
    K = np.block([[Q, A.T], [A, np.zeros((q.m, q.m))]])
    sol = np.linalg.solve(K, np.concatenate([-q.c, q.b]))
    g = _gpu_solve(q, tol=1e-9)
    assert g.status == P.OPTIMAL
    assert np.abs(g.x - sol[: q.n]).max() <= 1e-6 * (1 + np.abs(sol).max())


@pytest.mark.parametrize("inst", range(3))
def test_lp_matches_highs(torch, inst):
    q = I.tiny_lp(inst)
    A = q.A.toarray()
    lc, uc = _lc_uc(q)
    eq = lc == uc
    A_ub = np.vstack([A[~eq & np.isfinite(uc)], -A[~eq & np.isfinite(lc)]])
    b_ub = np.concatenate([uc[~eq & np.isfinite(uc)], -lc[~eq & np.isfinite(lc)]])
    ref = linprog(q.c, A_ub=A_ub, b_ub=b_ub, A_eq=A[eq], b_eq=lc[eq], bounds=_box(q.lb, q.ub),
                  method="highs")
    g = _gpu_solve(q, tol=1e-8, max_iter=400000)
    assert g.status == P.OPTIMAL
    assert g.info["primal_obj"] == pytest.approx(ref.fun, rel=1e-6, abs=1e-6)


def test_mixed_bounds_matches_oracle(torch):
    q = I.mixed_bounds(0)
    g = _gpu_solve(q, tol=1e-8)
    o = oracle.solve(q, tol=1e-8)
    assert g.status == o.status == P.OPTIMAL
    _assert_kkt(q, g, 1e-8)
    assert g.info["primal_obj"] == pytest.approx(o.info["primal_obj"], rel=1e-7, abs=1e-7)
    assert np.abs(g.x - o.x).max() <= 1e-4


def test_portfolio_diagonal_path_matches_oracle(torch):
    q = I.portfolio(0, n_assets=20000, k_factors=100)
    g = _gpu_solve(q)
    o = oracle.solve(q)
    assert g.status == o.status == P.OPTIMAL
    _assert_kkt(q, g)
    ref = oracle.solve(q, tol=1e-9, max_iter=400000)
    assert ref.status == P.OPTIMAL
    _assert_objective(g.info["primal_obj"], ref.info["primal_obj"], q.name)


def _separation(q, ray):
    A = q.A.toarray()
    lc, uc = _lc_uc(q)
    lo = linprog(A.T @ ray, bounds=_box(q.lb, q.ub), method="highs")
    hi = linprog(-ray, bounds=_box(lc, uc), method="highs")
    return lo.fun, -hi.fun


@pytest.mark.parametrize("make", ["contradictory", "box", "random_small"])
def test_primal_infeasible_matches_oracle(torch, make):
    q = {"contradictory": lambda: I.contradictory_rows(0), "box": lambda: I.box_infeasible_rows(0),
         "random_small": lambda: I.random_small(0, infeasible=True)}[make]()
    g = _gpu_solve(q, max_iter=20000)
    o = oracle.solve(q, max_iter=20000)
    assert g.status == o.status == P.PRIMAL_INFEASIBLE
    assert np.abs(g.y).max() == pytest.approx(1.0)
    inf_x, sup_s = _separation(q, g.y)
    assert inf_x > sup_s + 1e-9


def test_unbounded_matches_oracle(torch):
    q = I.unbounded_qp(0)
    g = _gpu_solve(q, max_iter=20000)
    o = oracle.solve(q, max_iter=20000)
    assert g.status == o.status == P.DUAL_INFEASIBLE
    d = g.x
    assert np.abs(d).max() == pytest.approx(1.0)
    assert np.abs(q.A @ d).max() <= 1e-8 and np.abs(q.Q @ d).max() <= 1e-8 and q.c @ d < 0


def test_iteration_limits_and_start_point(torch):
    q = I.random_small(0)
    g0 = _gpu_solve(q, max_iter=0)
    o0 = oracle.solve(q, max_iter=0)
    assert g0.status == o0.status == P.ITERATION_LIMIT and g0.info["iterations"] == 0
    assert np.array_equal(g0.x, o0.x) and np.all(g0.y == 0)
    for k in ("r_primal", "r_gap"):
        assert g0.info[k] == pytest.approx(o0.info[k], rel=1e-12)
    g1 = _gpu_solve(q, max_iter=1)
    assert g1.status == P.ITERATION_LIMIT and g1.info["iterations"] == 1


@pytest.mark.parametrize("every", [3, 64])
def test_general_q_iterates_match_oracle(torch, every):
    """The MPRGP path after a fixed number of iterations, with checks every
    3 (many restarts, the round's step count reset by the check's posted
    decision) or every 64 iterations: the same inner and restart counts as
    the oracle and the same iterates up to rounding order."""
    q = I.random_small(0)
    g = _gpu_solve(q, max_iter=150, check_every=every)
    o = oracle.solve(q, max_iter=150, check_every=every)
    assert g.status == o.status
    for key in ("iterations", "inner_iterations", "restarts"):
        assert g.info[key] == o.info[key], key
    for a, r, what in ((g.x, o.x, "x"), (g.y, o.y, "y")):
        err = np.abs(a - r).max() / (1.0 + np.abs(r).max())
        print(f"every {every}: {what} max relative difference {err:.2e}, restarts {g.info['restarts']}, "
              f"inner {g.info['inner_iterations']}", flush=True)
        assert err <= 1e-10, (what, err)


def test_no_rows_and_lp(torch):
    q = I.tiny(21, n=5, m=1)
    q.A = q.A[:0]
    q.b = q.b[:0]
    q.sense = b""
    q.m = 0
    g = _gpu_solve(q, tol=1e-9)
    o = oracle.solve(q, tol=1e-9)
    assert g.status == o.status == P.OPTIMAL
    assert np.abs(g.x - o.x).max() <= 1e-6
    lp = I.tiny_lp(5)
    g = _gpu_solve(lp, tol=1e-8, max_iter=400000)
    o = oracle.solve(lp, tol=1e-8, max_iter=400000)
    assert g.status == o.status == P.OPTIMAL
    assert g.info["primal_obj"] == pytest.approx(o.info["primal_obj"], rel=1e-6, abs=1e-6)


# ---- the 1e6-variable workload at full size ---------------------------------------

@pytest.fixture(scope="module")
def large():
    return I.large_sparse(0)


def test_large_spmv_sampled_rows(torch, large):
    q = large
    rng = np.random.default_rng(11)
    h = P.qp_create_from(q)
    try:
        for op, M, ncol in ((P.OP_Q, q.Q, q.n), (P.OP_A, q.A, q.n), (P.OP_AT, q.A.T.tocsr(), q.m)):
            x = rng.normal(size=ncol)
            yd = torch.zeros(M.shape[0], dtype=torch.float64, device="cuda")
            P.qp_apply(h, op, _dev(torch, x), yd)
            y = yd.cpu().numpy()
            rows = np.sort(rng.choice(M.shape[0], size=3000, replace=False))
            sub = M[rows]
            ref = oracle.matvec(sub, x)
            scale = abs(sub) @ np.abs(x)
            assert np.all(np.abs(y[rows] - ref) <= 1e-12 * scale + 1e-300)
    finally:
        P.qp_destroy(h)


def test_large_solve_kkt(torch, large):
    """The headline workload at full size: the oracle's status, relative KKT
    <= 1e-6 evaluated by the oracle on the returned point, and the objective
    of the oracle run at tol 1e-7 (stored) to the acceptance bound."""
    q = large
    gold = _golden("oracle_large_sparse_n1e6.json")["result"]
    assert (gold["n"], gold["m"], gold["nnz_Q"], gold["nnz_A"]) == (q.n, q.m, q.nnz_Q, q.nnz_A)
    g = _gpu_solve(q)
    print(f"large: status={g.status_name} iterations={g.info['iterations']} "
          f"inner={g.info['inner_iterations']} seconds={g.info['solve_seconds']:.2f}; oracle at tol "
          f"{gold['tol']}: {gold['status_name']} {gold['iterations']}/{gold['inner_iterations']} iterations")
    assert g.status == gold["status"] == P.OPTIMAL
    k = _assert_kkt(q, g)
    # y in Y: '>=' rows (second half) carry y <= 0
    assert np.all(g.y[q.m // 2:] <= 0)
    assert g.info["primal_obj"] == pytest.approx(k["pobj"], rel=1e-12)
    _assert_objective(g.info["primal_obj"], gold["primal_obj"], q.name)
    xs = _golden("oracle_large_sparse_n1e6.json")["x_sample"]
    dx = np.abs(g.x[np.asarray(xs["index"])] - np.asarray(xs["value"])).max()
    print(f"large: max |x - x_oracle| over {len(xs['index'])} sampled entries {dx:.2e}", flush=True)


def _p_support(z, l, u):
    """p(z; l, u) = u'z+ - l'z- (Section 2), summed exactly; a bound that is
    infinite where its part of z is zero contributes nothing."""
    zp, zm = np.maximum(z, 0.0), np.maximum(-z, 0.0)
    if np.any((zp > 0) & np.isinf(u)) or np.any((zm > 0) & np.isinf(l)):
        return math.inf, math.inf
    terms = np.concatenate([u[zp > 0] * zp[zp > 0], -l[zm > 0] * zm[zm > 0]])
    return math.fsum(terms.tolist()), float(np.abs(terms).sum())


def test_large_infeasible_variant(torch):
    """The infeasible variant at full size: the oracle's status (stored), and
    the returned ray satisfies Section 5.1's certificate, evaluated here from
    its definition: y~ in Y, A'y~ in R up to eps_inf times the improvement,
    and a strictly negative p(-A'y~; l_v, u_v) + p(y~; l_c, u_c)."""
    q = I.large_sparse(0, infeasible=True)
    gold = _golden("oracle_large_sparse_n1e6_infeasible.json")["result"]
    g = _gpu_solve(q, max_iter=20000)
    print(f"large infeasible: {g.status_name} after {g.info['iterations']} iterations; oracle "
          f"{gold['status_name']} after {gold['iterations']}", flush=True)
    assert g.status == gold["status"] == P.PRIMAL_INFEASIBLE
    r1, r2 = q.meta["rows"]
    assert sorted([r1, r2]) == sorted(gold["contradictory_rows"])
    top = set(np.argsort(-np.abs(g.y))[:2])
    assert top == {r1, r2} and g.y[r1] * g.y[r2] < 0
    yt = g.y
    lc, uc = _lc_uc(q)
    # y~ in Y: zero where both row bounds are infinite, <= 0 with only a
    # lower bound, >= 0 with only an upper bound
    assert np.all(yt[np.isinf(lc) & np.isinf(uc)] == 0)
    assert np.all(yt[np.isfinite(lc) & np.isinf(uc)] <= 0)
    assert np.all(yt[np.isinf(lc) & np.isfinite(uc)] >= 0)
    assert np.abs(yt).max() == pytest.approx(1.0)
    w = q.A.T.tocsr() @ yt
    # proj_R(w): R_i is {0} for a free variable, R- with only an upper bound,
    # R+ with only a lower bound, R for a boxed one
    lo_f, up_f = np.isfinite(q.lb), np.isfinite(q.ub)
    pw = np.where(lo_f & up_f, w, np.where(lo_f, np.maximum(w, 0), np.where(up_f, np.minimum(w, 0), 0.0)))
    viol = float(np.abs(w - pw).max())
    p1, a1 = _p_support(-w, q.lb, q.ub)
    p2, a2 = _p_support(yt, lc, uc)
    improvement = max(-(p1 + p2), 0.0)
    print(f"large infeasible: p(-A'y) + p(y) = {p1 + p2:.6e} (terms of total magnitude {a1 + a2:.3e}); "
          f"A'y violation of R {viol:.2e}", flush=True)
    assert improvement > 1e-9 * (a1 + a2)
    assert viol <= 1e-8 * improvement


@pytest.mark.parametrize("make", [lambda: I.random_small(0), lambda: I.mixed_bounds(0),
                                  lambda: I.random_factored(1, n=600, m=200, k=30)])
def test_graph_inner_steps_match_eager(torch, make):
    """The inner steps launched as captured graphs (2 or 5 steps per graph,
    replayed many times, eager launches in between) give the eager launches'
    result bit for bit, in FP64 and in mixed precision, over repeated solves."""
    q = make()
    with P.Solver(q) as s:
        for prec in (P.PRECISION_FP64, P.PRECISION_MIXED):
            ref = s.solve(graph_steps=0, precision=prec)
            for k in (2, 5, 2):
                g = s.solve(graph_steps=k, precision=prec)
                assert g.status == ref.status
                assert g.info["iterations"] == ref.info["iterations"]
                assert g.info["inner_iterations"] == ref.info["inner_iterations"]
                assert np.array_equal(g.x, ref.x) and np.array_equal(g.y, ref.y)


@pytest.mark.parametrize("make", [lambda: I.random_small(1),                 # one (l, u) pair
                                  lambda: I.mixed_bounds(0),                 # class table
                                  lambda: I.portfolio(1, n_assets=20000, k_factors=100),
                                  lambda: I.mixed_bounds(1, n=1200, m=400)])  # > 256 pairs: arrays
def test_bound_storage_gives_the_same_bits(torch, make, monkeypatch):
    """The box is stored as one pair, a byte class per variable, or arrays,
    whichever is smallest; every storage must give the same result bit for
    bit as the arrays."""
    q = make()
    g = _gpu_solve(q)
    monkeypatch.setenv("PDHCG_BOUND_STORAGE", "arrays")
    a = _gpu_solve(q)
    print(f"{q.name}: {g.info['iterations']}/{g.info['inner_iterations']} iterations, "
          f"{g.info['solve_seconds'] * 1e3:.1f} ms vs {a.info['solve_seconds'] * 1e3:.1f} ms with arrays")
    assert g.status == a.status == P.OPTIMAL
    assert g.info["iterations"] == a.info["iterations"]
    assert g.info["inner_iterations"] == a.info["inner_iterations"]
    assert np.array_equal(g.x, a.x) and np.array_equal(g.y, a.y)
    _assert_kkt(q, g)


def test_gather_rate_measurement(torch):
    """The gather-rate utility runs and gives a rate between the product's
    and a bound no device reaches (one gather per clock per CU at 3 GHz)."""
    g = P.measure_gather_rate(1_000_000, 11_000_000, 5)
    print(f"gather rate {g / 1e9:.0f} G/s", flush=True)
    assert 10e9 < g < 256 * 3e9 * 4
    with pytest.raises(P.QPError):
        P.measure_gather_rate(2, 11_000_000, 5)


def test_diagonal_q_with_dense_column_matches_oracle(torch):
    """Diagonal Q and a column of A in every row (A' has a row longer than a
    row block, completed in the closed-form step's own finishing kernel, so
    that step's finishing work is not carried into the dual step's)."""
    rng = np.random.default_rng(21)
    n, m = 3000, 2600
    A = sp.random(m, n, density=3.0 / n, random_state=rng, data_rvs=rng.standard_normal).tolil()
    A[:, 0] = 0.05 * rng.normal(size=(m, 1))
    A = sp.csr_matrix(A)
    A.sort_indices()
    x0 = rng.uniform(-0.5, 0.5, size=n)
    q = I.QP(n=n, m=m, Q=sp.diags(rng.uniform(0.5, 2.0, size=n)).tocsr(), A=A, c=rng.normal(size=n),
             b=A @ x0 - 0.05, sense=bytes([ord("G")] * m),
             lb=np.full(n, -1.0), ub=np.full(n, 1.0), name="dense_column")
    assert np.diff(sp.csc_matrix(A).indptr).max() > 2048
    g = _gpu_solve(q)
    o = oracle.solve(q)
    assert g.status == o.status == P.OPTIMAL
    _assert_kkt(q, g)
    ref = oracle.solve(q, tol=1e-9, max_iter=400000)
    _assert_objective(g.info["primal_obj"], ref.info["primal_obj"], q.name)
