"""The closed-form (diagonal Q) path when A has rows longer than a row
block.  In the iterations whose reductions nothing reads, the dual step
leaves those rows to the next primal kernel, and every block of that kernel
completes them from their segment partials before it gathers y.

Rows longer than 8192 nonzeros are split into segments.  The instance has
both kinds of segmented row:
- a dense row of 20 segments, summed by the whole block;
- forty rows of 5 or 6 segments, summed one thread per row.
It also has rows of 2100 to 4000 nonzeros, which one block sums in strided
passes.

Checked against the oracle in two ways.  The iterates after a fixed number
of iterations must agree, since both sides do the same arithmetic up to
rounding order.  The solve must return the oracle's status, KKT and
objective, in FP64 and in mixed precision.
"""

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
    T.cuda.init()
    return T


def _long_rows_qp(seed=5, n=40000):
    rng = np.random.default_rng(seed)
    cols, vals = [], []
    for _ in range(40):                      # 5 or 6 segments each
        j = np.sort(rng.choice(n, size=int(rng.integers(8500, 12000)), replace=False))
        cols.append(j)
        vals.append(rng.normal(size=j.size) / np.sqrt(j.size / 100.0))
    for _ in range(6):                       # one block's strided passes
        j = np.sort(rng.choice(n, size=int(rng.integers(2100, 4000)), replace=False))
        cols.append(j)
        vals.append(rng.normal(size=j.size) / np.sqrt(j.size / 100.0))
    cols.append(np.arange(n))                # dense row: 20 segments
    vals.append(rng.uniform(0.5, 1.5, size=n))
    for _ in range(9):                       # short rows
        j = np.sort(rng.choice(n, size=20, replace=False))
        cols.append(j)
        vals.append(rng.normal(size=j.size))
    m = len(cols)
    indptr = np.concatenate([[0], np.cumsum([c.size for c in cols])])
    A = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), indptr), shape=(m, n))
    x0 = rng.uniform(-0.5, 0.5, size=n)
    ne = m // 2
    sense = bytes([ord("E")] * ne + [ord("G")] * (m - ne))
    b = A @ x0
    b[ne:] -= rng.uniform(0.0, 0.1, size=m - ne)
    return I.QP(n=n, m=m, Q=sp.diags(rng.uniform(0.5, 2.0, size=n)).tocsr(), A=A, c=rng.normal(size=n),
                b=b, sense=sense, lb=np.full(n, -1.0), ub=np.full(n, 1.0), name="long_rows")


@pytest.fixture(scope="module")
def qp():
    q = _long_rows_qp()
    lens = np.diff(q.A.indptr)
    assert (lens > 8192).sum() == 41 and ((lens > 2048) & (lens <= 8192)).sum() == 6
    assert lens.max() > 8 * 2048
    return q


@pytest.mark.parametrize("iters", [9, 70, 200])
def test_iterates_match_oracle(torch, qp, iters):
    """Iteration limits that leave long rows to the primal kernel in most
    iterations: 9 covers the first round only; 70 and 200 also cross checks."""
    with P.Solver(qp) as s:
        g = s.solve(max_iter=iters)
    o = oracle.solve(qp, max_iter=iters)
    assert g.status == o.status == P.ITERATION_LIMIT
    assert g.info["iterations"] == o.info["iterations"] == iters
    for a, r, what in ((g.x, o.x, "x"), (g.y, o.y, "y")):
        err = np.abs(a - r).max() / (1.0 + np.abs(r).max())
        print(f"{iters} iterations: {what} max relative difference {err:.2e}", flush=True)
        assert err <= 1e-9, (what, err)


@pytest.mark.parametrize("every", [2, 3, 5])
def test_iterates_match_oracle_short_rounds(torch, qp, every):
    """Checks every 2, 3 or 5 iterations: rounds of one or a few steps that
    leave long rows, restarts that reset the round right after a completion,
    and the full finishing kernel before every check, in quick alternation."""
    with P.Solver(qp) as s:
        g = s.solve(max_iter=150, check_every=every)
    o = oracle.solve(qp, max_iter=150, check_every=every)
    assert g.status == o.status
    assert g.info["iterations"] == o.info["iterations"]
    assert g.info["restarts"] == o.info["restarts"]
    for a, r, what in ((g.x, o.x, "x"), (g.y, o.y, "y")):
        err = np.abs(a - r).max() / (1.0 + np.abs(r).max())
        print(f"check every {every}: {what} max relative difference {err:.2e}, "
              f"restarts {g.info['restarts']}", flush=True)
        assert err <= 1e-9, (what, err)


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_solve_matches_oracle(torch, qp, precision):
    with P.Solver(qp) as s:
        g = s.solve(precision=precision)
    o = oracle.solve(qp)
    assert g.status == o.status == P.OPTIMAL
    k = oracle.kkt(qp, g.x, g.y)
    assert max(k["r_primal"], k["r_dual"], k["r_gap"]) <= 1e-6, k
    ref = oracle.solve(qp, tol=1e-9, max_iter=400000)
    assert ref.status == P.OPTIMAL
    err = abs(g.info["primal_obj"] - ref.info["primal_obj"]) / (1 + abs(ref.info["primal_obj"]))
    print(f"precision {precision}: objective error {err:.2e}, iterations {g.info['iterations']}", flush=True)
    assert err <= 1e-6
