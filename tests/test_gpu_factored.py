"""Q = P + R'R given by its factors (the structured quadratic objective):
the GPU's matrix-free product and solves against the oracle run on Q
written out."""

import json
import os

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


def _kkt_max(q, x, y):
    k = oracle.kkt(q, x, y)
    return max(k["r_primal"], k["r_dual"], k["r_gap"])


def test_factored_product_matches_explicit(torch):
    q = I.random_factored(0)
    Qe = q.explicit_Q()
    rng = np.random.default_rng(3)
    h = P.qp_create_from(q)
    try:
        for _ in range(3):
            x = rng.normal(size=q.n)
            yd = torch.zeros(q.n, dtype=torch.float64, device="cuda")
            P.qp_apply(h, P.OP_Q, torch.from_numpy(x).cuda(), yd)
            y = yd.cpu().numpy()
            ref = oracle.matvec(Qe, x)
            scale = abs(Qe) @ np.abs(x)
            assert np.all(np.abs(y - ref) <= 1e-12 * scale + 1e-300)
    finally:
        P.qp_destroy(h)


@pytest.mark.parametrize("make", [
    lambda: I.random_factored(0),
    lambda: I.random_factored(1, n=600, m=200, k=30),
    lambda: I.random_factored(2, boxed=False),
    lambda: I.portfolio_factored(3, n_assets=3000, k_factors=30),
])
def test_factored_solve_matches_oracle(torch, make):
    q = make()
    e = q.explicit()
    with P.Solver(q) as s:
        g = s.solve()
    o = oracle.solve(e, max_iter=400000)
    assert g.status == o.status == P.OPTIMAL, (g.status_name, o.status_name)
    assert _kkt_max(e, g.x, g.y) <= 1e-6
    ref = oracle.solve(e, tol=1e-9, max_iter=400000)
    f, fr = g.info["primal_obj"], ref.info["primal_obj"]
    print(f"{q.name}: it {g.info['iterations']}/{g.info['inner_iterations']} obj err "
          f"{abs(f - fr) / (1 + abs(fr)):.2e}")
    assert abs(f - fr) <= 1e-6 * (1 + abs(fr))


@pytest.mark.parametrize("every", [3, 64])
def test_factored_iterates_match_oracle(torch, every):
    """Q given as P + R'R (never formed) against the oracle on the explicit
    Q, after 150 iterations: the same inner and restart counts, the same
    iterates up to the order of the products' sums."""
    q = I.random_factored(0)
    e = q.explicit()
    with P.Solver(q) as s:
        g = s.solve(max_iter=150, check_every=every)
    o = oracle.solve(e, max_iter=150, check_every=every)
    assert g.status == o.status
    for key in ("iterations", "inner_iterations", "restarts"):
        assert g.info[key] == o.info[key], key
    for a, r, what in ((g.x, o.x, "x"), (g.y, o.y, "y")):
        err = np.abs(a - r).max() / (1.0 + np.abs(r).max())
        print(f"every {every}: {what} max relative difference {err:.2e}, restarts {g.info['restarts']}, "
              f"inner {g.info['inner_iterations']}", flush=True)
        assert err <= 1e-10, (what, err)


def test_factored_mixed_precision(torch):
    q = I.random_factored(4)
    e = q.explicit()
    with P.Solver(q) as s:
        g = s.solve(precision=P.PRECISION_MIXED)
    assert g.status == P.OPTIMAL
    assert _kkt_max(e, g.x, g.y) <= 1e-6
    ref = oracle.solve(e, tol=1e-9, max_iter=400000)
    assert abs(g.info["primal_obj"] - ref.info["primal_obj"]) <= 1e-6 * (1 + abs(ref.info["primal_obj"]))


def test_factored_portfolio_full_size_agrees_with_factor_variables(torch):
    """200k assets, 1000 factors: the factored form (CG inner solve, one row)
    and the factor-variable form (closed form, 1001 rows) reach the same
    optimum on the GPU, and both match the objective of the oracle run on
    the factor-variable form at tol 1e-9 (stored; the two forms have the same
    optimal objective) to 1e-6 (1 + |f|)."""
    qf = I.portfolio_factored(0)
    qv = I.portfolio(0)
    with P.Solver(qf) as s:
        gf = s.solve()
    with P.Solver(qv) as s:
        gv = s.solve()
    assert gf.status == gv.status == P.OPTIMAL
    f, fv = gf.info["primal_obj"], gv.info["primal_obj"]
    print(f"factored: {gf.info['iterations']}/{gf.info['inner_iterations']} it "
          f"{gf.info['solve_seconds'] * 1e3:.0f} ms; factor variables: {gv.info['iterations']} it "
          f"{gv.info['solve_seconds'] * 1e3:.0f} ms; obj diff {abs(f - fv) / (1 + abs(fv)):.2e}")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_portfolio_200k.json")) as fh:
        gold = json.load(fh)["result"]
    fr = gold["primal_obj"]
    for tag, val in (("factored", f), ("factor variables", fv)):
        err = abs(val - fr) / (1 + abs(fr))
        print(f"{tag}: objective error vs the oracle at tol 1e-9 {err:.2e}")
        assert err <= 1e-6
    assert np.abs(gf.x - gv.x[: qf.n]).max() <= 1e-4
