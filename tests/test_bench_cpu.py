"""Host-side logic of bench.py: the algorithmic byte counts behind the
roofline figures, the bound-storage rule they mirror, and the one-GPU guard."""

import subprocess
import sys
import os

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2602_23967_amd import instances as I  # noqa: E402


def _qp(lb, ub, n=6):
    return I.QP(n=n, m=1, Q=None, A=sp.csr_matrix(np.ones((1, n))), c=np.zeros(n), b=np.zeros(1),
                sense=b"E", lb=np.asarray(lb, dtype=float), ub=np.asarray(ub, dtype=float))


def test_bound_bytes_rule():
    # one shared pair: nothing per variable
    assert bench.bound_bytes(_qp([0.0] * 6, [10.0] * 6)) == 0
    # a few distinct pairs: a class byte per variable
    assert bench.bound_bytes(_qp([0, 0, -1, -1, -np.inf, 0], [1, 1, 1, 1, np.inf, 1])) == 1
    # more than 256 distinct pairs: two FP64 arrays
    n = 300
    assert bench.bound_bytes(_qp(-np.arange(n, dtype=float), np.ones(n), n=n)) == 16
    # -0.0 and 0.0 are different bit patterns, so different classes
    assert bench.bound_bytes(_qp([0.0, -0.0], [1.0, 1.0], n=2)) == 1


def test_hp_bytes_counts():
    n, nnz = 1000, 11000
    # 12 B per nonzero, int32 row pointers, p gathered once, g and x read,
    # H p written, the box by its storage
    assert bench.hp_bytes(n, nnz, 0) == 12 * nnz + 4 * (n + 1) + 8 * n * 4
    assert bench.hp_bytes(n, nnz, 16) - bench.hp_bytes(n, nnz, 0) == 16 * n
    # the large sparse instance's figure quoted in the design notes
    assert bench.hp_bytes(1_000_000, 10_999_950, 0) == 167_999_404


def test_batch_bytes_counts():
    q = I.mpc(0)
    per = bench.batch_bytes(q, 1, 6, 1)
    assert per == 2 * 6 * q.nnz_A + 4 * (q.n + q.m + 2) + 8 * q.n * 10 + 1 * q.n + 8 * q.m * 6
    assert bench.batch_bytes(q, 7, 6, 1) == 7 * per


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _served_results(qs):
    """Stand-ins for the server's results: the oracle's own solutions (the
    check below must accept them)."""
    import types
    import oracle
    res = []
    for q in qs:
        o = oracle.solve(q, tol=1e-9, max_iter=1_000_000)
        g = types.SimpleNamespace(status=o.status, x=o.x.copy(), y=o.y.copy(),
                                  info={"primal_obj": o.info["primal_obj"]})
        res.append((g, {}))
    return res


def test_verify_served_accepts_and_flags():
    """The served stream's oracle check: a seeded 5 % sample plus every
    infeasible request; agreeing results verify, a planted objective error
    or a wrong status is reported as a mismatch."""
    import types
    import paper_2602_23967_amd as P
    qs = [I.tiny(i) for i in range(19)] + [I.random_small(7, n=200, infeasible=True)]
    args = types.SimpleNamespace(verify_budget_s=120.0, tol=1e-6)
    res = _served_results(qs)
    v = bench.verify_served(qs, res, args, P)
    assert v["selected"] == 2 and v["checked"] == 2 and v["verified"] == 2, v
    assert v["mismatches"] == [] and v["single_thread"] is None
    args1 = types.SimpleNamespace(verify_budget_s=120.0, tol=1e-6, verify_single_thread=True)
    v1 = bench.verify_served(qs, res, args1, P)
    assert v1["verified"] == 2 and v1["single_thread"]["requests"] == 2
    assert v1["single_thread"]["cores"] == 1
    assert res[19][0].status == P.PRIMAL_INFEASIBLE
    # the sampled request (the one that is not the infeasible one)
    rng = np.random.default_rng(bench.SERVE_VERIFY_SEED)
    picked = int(rng.choice(len(qs), size=1, replace=False)[0])
    assert picked != 19
    g = res[picked][0]
    assert g.status == P.OPTIMAL
    g.info["primal_obj"] += 1e-3 * (1 + abs(g.info["primal_obj"]))
    res[19][0].status = P.OPTIMAL
    v = bench.verify_served(qs, res, args, P)
    assert v["verified"] == 0 and len(v["mismatches"]) == 2
    assert {r["request"] for r in v["mismatches"]} == {picked, 19}


def test_summary_keeps_served_figures():
    out = {"value": 5.0, "unit": "QPs solved/s", "ms_per_step": 1.0, "steps": 1, "dtype": "f64",
           "solved": 9, "requests": 10, "latency_s": {"p50": 0.1, "p99": 1.0, "per_kind": {}},
           "one_at_a_time": {"value": 1.0}, "oracle_verified": {"checked": 2, "verified": 2},
           "roofline": None, "config": {"workload": "served stream", "batch_lanes": 2}}
    s = bench.summary(out)
    assert s["workload"] == "served stream"
    assert s["oracle_verified"] == {"checked": 2, "verified": 2}
    assert s["requests"] == 10 and s["latency_s"]["p99"] == 1.0
    assert "roofline" not in s and "batch_lanes" not in s


def test_measured_full_solve_record():
    """The stored whole-solve record is read back for its own workload and
    tolerance only, and its figures agree with the summary beside it."""
    r = bench.measured_full_solve("large_sparse", 1e-6)
    assert r is not None and r["status"] == "OPTIMAL"
    assert r["value"] == pytest.approx(1.0 / r["seconds"])
    assert r["command"].startswith("python3 bench.py --cpu-full")
    md = open(os.path.join(ROOT, "profiles", "cpu_oracle_large_sparse_n1e6.md")).read()
    assert f"{r['seconds']} s" in md and f"{r['inner_iterations']:,} inner" in md
    assert bench.measured_full_solve("large_sparse", 1e-4) is None
    assert bench.measured_full_solve("portfolio", 1e-6) is None
