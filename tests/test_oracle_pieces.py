"""Pins of the oracle's small pieces against facts that do not come from the
oracle itself: published constants and test vectors, closed forms, and
algebraic identities of the sets of Section 2."""

import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import oracle
from paper_2602_23967_amd import instances as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_constants_are_defaults():
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    p = oracle.params()
    assert p.gamma_inner == g["gamma_inner"]["value"]
    assert p.eps_min == g["eps_min"]["value"]
    assert p.eta_scale == g["eta_scale"]["value"]
    assert p.tol == g["tol"]["value"]


def test_splitmix_published_vector():
    g = json.load(open(os.path.join(GOLD, "splitmix64_seed0.json")))
    for i, h in enumerate(g["outputs_hex"]):
        want = (int(h, 16) >> 11) * 2.0 ** -53
        assert oracle.splitmix_unit(i) == want


def test_bounds_from_sense():
    lc, uc = oracle.bounds_from_sense(np.array([1.0, 2.0, 3.0]), b"EGL")
    assert list(lc) == [1.0, 2.0, -np.inf]
    assert list(uc) == [1.0, np.inf, 3.0]
    with pytest.raises(ValueError):
        oracle.bounds_from_sense(np.array([1.0]), b"X")


# ---- support function p(z; l, u) = max over the box of z's inner product ----

def _box_max(z, l, u):
    """sup_{l<=s<=u} z's by linear programming (independent of the oracle)."""
    from scipy.optimize import linprog
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
              for a, b in zip(l, u)]
    r = linprog(-z, bounds=bounds, method="highs")
    if r.status == 3:
        return np.inf
    return -r.fun


@settings(max_examples=60, deadline=None)
@given(st.lists(st.tuples(st.floats(-5, 5), st.floats(0, 3), st.sampled_from([0, 1, 2, 3])),
                min_size=1, max_size=6))
def test_support_is_box_maximum(items):
    """p(z; l, u) = u'z+ - l'z- is the support function of [l, u]: it equals
    max_{s in [l,u]} z's, which an LP computes independently."""
    z = np.array([a for a, _, _ in items])
    z = np.where(np.abs(z) < 1e-3, 0.0, z)     # stay clear of the LP solver's 1e-7 tolerances
    l = np.array([-w if k in (0, 1) else -np.inf for _, w, k in items])
    u = np.array([w + 0.5 if k in (0, 2) else np.inf for _, w, k in items])
    # keep z in the set where p is finite (the dual cone of the box)
    z = np.where(~np.isfinite(u) & (z > 0), 0.0, z)
    z = np.where(~np.isfinite(l) & (z < 0), 0.0, z)
    assert oracle.support(z, l, u) == pytest.approx(_box_max(z, l, u), rel=1e-12, abs=1e-12)


def test_support_zero_times_infinity_is_zero():
    assert oracle.support(np.array([0.0, 0.0]), np.array([-np.inf, 1.0]),
                          np.array([np.inf, 2.0])) == 0.0
    assert oracle.support(np.array([1.0]), np.array([-1.0]), np.array([np.inf])) == np.inf


# ---- power iteration ---------------------------------------------------------

@pytest.mark.parametrize("inst", [0, 1])
def test_norm2_matches_svd(inst):
    q = I.random_small(inst)
    exact = np.linalg.norm(q.A.toarray(), 2)
    est = oracle.norm2(q.A, tol=1e-10, max_iter=5000)
    assert est <= exact * (1 + 1e-12)          # Rayleigh quotient never overshoots
    assert est == pytest.approx(exact, rel=1e-6)
    # default tolerance with the 1% safety factor gives a safe step size
    est7 = oracle.norm2(q.A)
    assert 1.01 * est7 >= exact
    eta = 0.998 / (1.01 * est7)
    assert eta * eta * exact ** 2 < 1.0        # tau*sigma*||A||^2 < 1


def test_norm2_symmetric_q():
    q = I.random_small(0)
    lam = np.linalg.eigvalsh(q.Q.toarray()).max()
    assert oracle.norm2(q.Q, tol=1e-12, max_iter=20000) == pytest.approx(lam, rel=1e-6)


def test_norm2_zero_and_empty():
    Z = sp.csr_matrix((3, 4))
    assert oracle.norm2(Z) == 0.0


# ---- Halpern, PID, inner tolerance, restart: algebra on hand values ------------

def test_halpern_affine_and_special_cases():
    rng = np.random.default_rng(0)
    v = rng.normal(size=5)
    # weights sum to one: a fixed point shared with the anchor stays put
    for t in range(5):
        for th in (0.0, 0.5, 1.0):
            assert np.allclose(oracle.halpern(t, th, v, v, v), v, rtol=0, atol=1e-15)
    zt, z, za = rng.normal(size=(3, 5))
    # t = 0, theta = 0: midpoint of T(z) and the anchor
    assert np.allclose(oracle.halpern(0, 0.0, zt, z, za), 0.5 * zt + 0.5 * za, atol=1e-15)
    # t = 2, theta = 1: (3/4)(2 T(z) - z) + (1/4) anchor
    assert np.allclose(oracle.halpern(2, 1.0, zt, z, za), 0.75 * (2 * zt - z) + 0.25 * za,
                       atol=1e-15)


def test_pid_proportional_gain_one_hits_balance():
    """With K_P = 1 and no I/D term the update lands on the weight that makes
    sqrt(w)||dx|| = ||dy||/sqrt(w), i.e. w = ||dy||/||dx|| (Section 3.2)."""
    w, integ, prev = oracle.pid(2.0, 1.0, 0.5, 3.0, 1.0, 0.0, 0.0)
    assert w == pytest.approx(6.0, rel=1e-14)
    e = math.log(2.0 * 0.5 / 3.0)
    assert integ == pytest.approx(e) and prev == pytest.approx(e)


def test_pid_integral_and_derivative_terms():
    # two rounds by hand: e1 = log(1*2/1) = log 2 ; omega1 = exp(-(kp e1 + ki e1 + kd e1))
    kp, ki, kd = 0.5, 0.1, 0.2
    w1, i1, p1 = oracle.pid(1.0, 1.0, 2.0, 1.0, kp, ki, kd)
    e1 = math.log(2.0)
    assert w1 == pytest.approx(math.exp(-(kp * e1 + ki * e1 + kd * e1)))
    w2, i2, p2 = oracle.pid(w1, 1.0, 1.0, 1.0, kp, ki, kd, i1, p1)
    e2 = math.log(w1)
    assert w2 == pytest.approx(math.exp(math.log(w1) - (kp * e2 + ki * (e1 + e2) + kd * (e2 - e1))))


def test_pid_guards():
    assert oracle.pid(3.0, 1.0, 0.0, 1.0, 1, 0, 0)[0] == 3.0          # no primal movement
    assert oracle.pid(3.0, 1.0, 1.0, 1e-12, 1, 0, 0)[0] == 3.0        # no dual movement
    w = oracle.pid(1.0, 1.0, 1.0, 1e30, 1.0, 0, 0)[0]                  # clamped to omega0*e^10
    assert w == pytest.approx(math.exp(10.0))


def test_inner_tolerance_rule():
    g, emin = 5e-4, 1e-9
    # formula value when it lies between the floor and the previous tolerance
    assert oracle.inner_tol(1.0, g, 2.0, 0.5, 3.0, emin) == pytest.approx(g * 2.0 * 3.0 / 0.5)
    # monotone: never relaxes
    assert oracle.inner_tol(1e-4, g, 2.0, 0.5, 3.0, emin) == 1e-4
    # floor
    assert oracle.inner_tol(1.0, g, 1.0, 1.0, 0.0, emin) == emin
    eps = np.inf
    rng = np.random.default_rng(1)
    for _ in range(200):
        new = oracle.inner_tol(eps, g, rng.uniform(0.1, 10), rng.uniform(0.01, 1),
                               rng.exponential(), emin)
        assert emin <= new <= eps
        eps = new


def test_restart_rule():
    p = oracle.params()
    assert oracle.restart_test(0.19, 1.0, 0.5, True, 5, 1000, p)         # sufficient decay
    assert not oracle.restart_test(0.5, 1.0, 0.6, True, 5, 1000, p)      # still decaying
    assert oracle.restart_test(0.5, 1.0, 0.45, True, 5, 1000, p)         # necessary + stalled
    assert not oracle.restart_test(0.5, 1.0, 0.45, False, 5, 1000, p)    # no previous check
    assert oracle.restart_test(0.99, 1.0, 0.5, True, 360, 1000, p)       # artificial
    assert not oracle.restart_test(0.99, 1.0, 0.5, True, 359, 1000, p)
