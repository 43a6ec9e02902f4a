#!/usr/bin/env python3
"""Benchmark: QPs solved per second at 1e-6 relative KKT on one MI355X.

One step is one full solve (every outer PDHG iteration and every inner
conjugate-gradient iteration, on device) of the large sparse workload:
n = 1e6 variables, m = 5e5 rows (half '=', half '>='), Q symmetric with
about 10 random off-diagonals per row and a dominant diagonal, A with 8
nonzeros per row, box [0, 10], tolerance 1e-6.  The problem data is
resident in HBM before the timed region (qp_create runs first).

Prints one JSON line with the throughput, p50/p99 latency, the roofline
of the dominant kernel (measured with HIP events inside the timed solves)
and the CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QPs solved/s at 1e-6 rel KKT + achieved HBM GB/s; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
SERVE_VERIFY_SEED = 2602_23967
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_spmv_hp_large_sparse.json")
CPU_FULL_FILE = os.path.join(ROOT, "profiles", "cpu_oracle_large_sparse_n1e6.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernels_digest():
    h = hashlib.sha256()
    for f in ("kernels.hip", "pdhcg_internal.h", "schedule.h"):
        with open(os.path.join(ROOT, "paper_2602_23967_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bound_bytes(q):
    """Bytes per variable the kernels read for the box (l_v, u_v): 0 when
    every variable has the same pair, 1 (a class byte) for at most 256
    distinct pairs, 16 otherwise -- the library's storage rule."""
    lb = np.full(q.n, -np.inf) if q.lb is None else np.asarray(q.lb, dtype=np.float64)
    ub = np.full(q.n, np.inf) if q.ub is None else np.asarray(q.ub, dtype=np.float64)
    pairs = np.unique(np.stack([lb.view(np.uint64), ub.view(np.uint64)], axis=1), axis=0)
    return 0 if len(pairs) == 1 else (1 if len(pairs) <= 256 else 16)


def hp_bytes(n, nnz_q, bb=16):
    """Algorithmic HBM bytes of one launch of the inner H p kernel:
    CSR values and columns (12 B per nonzero), int32 row pointers, the
    gathered operand p once, the epilogue's reads of g and x and the write
    of Hp (8 B each per row), and the box (bb bytes per row, bound_bytes)."""
    return 12 * nnz_q + 4 * (n + 1) + 8 * n * 4 + bb * n


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(q, gpu_info, sample_iters, tol):
    """The oracle on the host cores, on a bounded sample: its first
    `sample_iters` outer iterations (with their inner solves and the check
    that ends the sample).  The oracle times its phases; the cost of one
    outer step (inner solve excluded), one inner step and one check is each
    applied to the GPU run's counts, so the estimate follows the full
    solve's mix of outer and inner steps (setup -- the norm estimates --
    excluded on both sides)."""
    import oracle

    t = time.perf_counter()
    r = oracle.solve(q, tol=tol, max_iter=sample_iters)
    wall = time.perf_counter() - t
    i = r.info
    per_inner = i["seconds_inner"] / max(i["inner_iterations"], 1)
    per_check = i["seconds_check"] / max(i["checks"], 1)
    per_outer = (i["seconds_total"] - i["seconds_setup"] - i["seconds_inner"] - i["seconds_check"]) / max(
        i["iterations"], 1)
    go, gi, gc = gpu_info["iterations"], gpu_info["inner_iterations"], gpu_info["checks"]
    est = per_outer * go + per_inner * gi + per_check * gc
    log(f"oracle sample {wall:.1f}s: {i['iterations']} outer ({per_outer * 1e3:.2f} ms each), "
        f"{i['inner_iterations']} inner ({per_inner * 1e3:.2f} ms each), {i['checks']} checks "
        f"({per_check * 1e3:.1f} ms each); full-solve estimate {est:.1f}s")
    return {
        "value": 1.0 / est,
        "unit": "QPs solved/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "method": "phase costs of a bounded sample applied to the GPU run's step counts",
        "sample": (f"oracle_qp_solve on the same instance for its first {i['iterations']} outer iterations "
                   f"({i['inner_iterations']} inner, {i['checks']} checks) in {wall:.2f}s, "
                   f"{i['seconds_setup']:.2f}s of it setup; per outer step {per_outer * 1e3:.3f} ms, per inner "
                   f"step {per_inner * 1e3:.3f} ms, per check {per_check * 1e3:.2f} ms, applied to "
                   f"{go} outer + {gi} inner steps + {gc} checks"),
    }


def measured_full_solve(workload, tol):
    """The oracle's whole solve of this workload, run to completion once
    with `--cpu-full` on the same host (minutes of CPU time, too long for
    the default run) and stored with the command that produced it.  It is
    reported beside the bounded-sample estimate, never in its place."""
    if not os.path.exists(CPU_FULL_FILE):
        return None
    with open(CPU_FULL_FILE) as f:
        rec = json.load(f)
    if rec.get("workload") != workload or rec.get("tol") != tol:
        return None
    return {"value": 1.0 / rec["seconds"], "unit": "QPs solved/s", "seconds": rec["seconds"],
            "cores": rec["cores"], "status": rec["status"], "iterations": rec["iterations"],
            "inner_iterations": rec["inner_iterations"], "primal_obj": rec["primal_obj"],
            "sample_estimate_seconds_same_run": rec["sample_estimate_seconds_same_run"],
            "source": os.path.relpath(CPU_FULL_FILE, ROOT), "command": rec["command"]}


def cpu_small(q, tol, budget_s=10.0):
    """Whole oracle solves of a small instance, repeated for about budget_s
    on all host threads and again on one thread."""
    import oracle
    nth = oracle.num_threads()
    res = {}
    for threads in (nth, 1):
        oracle.set_num_threads(threads)
        t = time.perf_counter()
        k = 0
        while k == 0 or time.perf_counter() - t < budget_s / 2:
            oracle.solve(q, tol=tol)
            k += 1
        res[threads] = (k, time.perf_counter() - t)
    oracle.set_num_threads(nth)
    (k, el), (k1, el1) = res[nth], res[1]
    return {"value": k / el, "unit": "QPs solved/s", "cores": nth, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{k} whole oracle_qp_solve runs of the same instance in {el:.2f}s",
            "single_thread": {"value": k1 / el1, "cores": 1,
                              "sample": f"{k1} whole runs in {el1:.2f}s"}}


def cpu_full(workload, tol, budget_s, threads=0):
    """The oracle's whole solve of a workload, run in a child process under
    its own time budget (a run past the budget is reported as a timeout)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", workload, "--tol", repr(tol)]
    env = dict(os.environ)
    if threads > 0:
        env["OMP_NUM_THREADS"] = str(threads)
    t = time.perf_counter()
    try:
        p = subprocess.run(cmd, capture_output=True, text=True, timeout=budget_s, env=env)
    except subprocess.TimeoutExpired:
        return {"timeout_s": budget_s, "kind": "oracle", "cpu_model": cpu_model()}
    el = time.perf_counter() - t
    if p.returncode != 0:
        raise RuntimeError(f"oracle child failed: {p.stderr[-2000:]}")
    res = json.loads(p.stdout.strip().splitlines()[-1])
    res.update({"kind": "oracle", "cpu_model": cpu_model(), "child_wall_s": el})
    return res


def oracle_child(workload, tol):
    """Body of the child process of cpu_full: generate, solve, print JSON."""
    import oracle
    from paper_2602_23967_amd import instances as I
    if workload == "large_sparse":
        qs = [I.large_sparse(0)]
    elif workload == "small":
        qs = [I.random_small(0)]
    elif workload == "portfolio":
        qs = [I.portfolio(0)]
    elif workload == "mpc_batch":
        qs = [I.mpc(i) for i in range(4096)]
    else:
        raise SystemExit(f"no oracle child for {workload}")
    t = time.perf_counter()
    st, it, inner, objs = [], 0, 0, []
    for q in qs:
        r = oracle.solve(q, tol=tol)
        st.append(r.status)
        it += r.info["iterations"]
        inner += r.info["inner_iterations"]
        objs.append(r.info["primal_obj"])
    el = time.perf_counter() - t
    out = {"workload": workload, "instances": len(qs), "seconds": el, "value": len(qs) / el,
           "unit": "QPs solved/s", "cores": oracle.num_threads(),
           "optimal": int(sum(s_ == oracle.OPTIMAL for s_ in st)), "iterations": it,
           "inner_iterations": inner}
    if len(qs) == 1:
        out["status"] = oracle.STATUS_NAMES[st[0]]
        out["primal_obj"] = objs[0]
    print(json.dumps(out), flush=True)


def batch_bytes(q, iters, vb=12, bb=16):
    """Algorithmic bytes of one instance's iterations in the batched kernel:
    the A and A' products (vb B per nonzero each: the value, 8 in FP64 or 4
    in FP32, and the column index, 2 when every instance is below 65536
    variables and rows (16-bit local indices) else 4; int32 row pointers),
    the primal step (x, c, q, l_v, u_v read; x_T, x_bar written), the dual
    step (x_bar gathered once; y, y anchor, l_c, u_c read; y_T, y written)
    and the Halpern step on x (x_T, x, anchor read; x written) -- counted
    as HBM traffic, as in the form that keeps no iterate on chip; the box
    costs bb bytes per variable (bound_bytes of the whole batch)."""
    per_iter = 2 * vb * q.nnz_A + 4 * (q.n + q.m + 2) + 8 * q.n * 10 + bb * q.n + 8 * q.m * 6
    return per_iter * iters


def main_batch(args, torch, P, I):
    t = time.perf_counter()
    qs = [I.mpc(i) for i in range(args.count)]
    log(f"generated {len(qs)} MPC instances in {time.perf_counter() - t:.1f}s "
        f"(n {sum(q.n for q in qs)}, m {sum(q.m for q in qs)}, nnz(A) {sum(q.nnz_A for q in qs)})")
    bs = P.BatchSolver(qs)
    mixed = args.precision == "mixed"
    params = P.qp_params_default(tol=args.tol, max_iter=args.max_iter,
                                 precision=P.PRECISION_MIXED if mixed else P.PRECISION_FP64)
    # launch schedule: the autotuner's pick (timed on these instances before
    # the warmup, outside the timed region), the library default, or given
    sched = {}
    if args.schedule == "auto":
        t = time.perf_counter()
        e = bs.tune(params)
        sched = {"source": "autotuner", "tune_s": time.perf_counter() - t,
                 "candidates_ms": [round(v * 1e3, 2) for v in e["seconds"]]}
        log(f"autotuner: shape {e['shape']} ({e['threads']} threads, {e['lds']} LDS doubles, "
            f"{e['waves_per_simd']} waves/SIMD), order {e['order']} in {sched['tune_s']:.1f}s; "
            f"candidates {sched['candidates_ms']} ms")
    elif args.schedule != "default":
        sh, od = (int(v) for v in args.schedule.split(","))
        bs.set_schedule(sh, od)
        sched = {"source": "given"}
    else:
        sched = {"source": "library default"}
    shape, order = bs.schedule()
    threads, lds, waves = P.qp_batch_shape_info(shape)
    sched.update({"shape": shape, "order": order, "threads": threads, "lds_doubles": lds,
                  "waves_per_simd": waves})
    for w in range(args.warmup):
        st, sec = bs.solve(params)
        log(f"warmup {w}: {int(np.sum(st == P.OPTIMAL))}/{len(qs)} optimal in {sec * 1e3:.1f} ms")
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        a = time.perf_counter()
        st, sec = bs.solve(params)
        lat.append(time.perf_counter() - a)
        log(f"step {s_}: {int(np.sum(st == P.OPTIMAL))}/{len(qs)} optimal in {lat[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # the last launch's per-instance times (device wall clock): when each
    # instance finished after the launch's first instance was taken up, and
    # how long its workgroup took over it
    t_take, t_done = bs.times()
    infos = [bs.result(i).info for i in range(len(qs))]
    iters = [i["iterations"] for i in infos]
    col_b = 2 if max(max(q.n, q.m) for q in qs) <= 65536 else 4
    whole = type("Box", (), {"n": sum(q.n for q in qs),
                             "lb": np.concatenate([np.full(q.n, -np.inf) if q.lb is None else q.lb for q in qs]),
                             "ub": np.concatenate([np.full(q.n, np.inf) if q.ub is None else q.ub for q in qs])})
    bb = bound_bytes(whole)
    nbytes = sum(batch_bytes(q, it, (4 if mixed else 8) + col_b, bb) for q, it in zip(qs, iters))
    kernel_s = float(np.median(lat))
    bs.close()
    # the same instances one at a time through the single-QP path, FP64
    one = []
    p64 = P.qp_params_default(tol=args.tol, max_iter=args.max_iter)
    for q in qs[: args.one_at_a_time]:
        with P.Solver(q) as s1:
            r = s1.solve(p64)
            one.append(r.info["solve_seconds"])
    # solved: OPTIMAL with the solver's own KKT at the tolerance (the tests
    # check these points with the oracle's KKT evaluation)
    n_ok = sum(1 for i in infos if i["status"] == P.OPTIMAL and
               max(i["r_primal"], i["r_dual"], i["r_gap"]) <= args.tol)
    out = {
        "metric": METRIC,
        "value": n_ok * args.steps / elapsed,
        "unit": "QPs solved/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products + f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"batched linear MPC, {len(qs)} instances, horizon T ~ U{{10..50}}, "
                               f"12 states, 4 inputs, one persistent launch, tol {args.tol:g}, "
                               f"{'mixed precision' if mixed else 'FP64'}",
                   "instances": len(qs)},
        "solved": bool(np.all(st == P.OPTIMAL)),
        "solved_count": int(n_ok),
        "instance_times_ms": {
            "completion_p50": 1e3 * float(np.percentile(t_done, 50)),
            "completion_p99": 1e3 * float(np.percentile(t_done, 99)),
            "completion_max": 1e3 * float(np.max(t_done)),
            "solve_p50": 1e3 * float(np.percentile(t_done - t_take, 50)),
            "solve_p99": 1e3 * float(np.percentile(t_done - t_take, 99)),
            "solve_max": 1e3 * float(np.max(t_done - t_take)),
            "note": "last timed launch; completion = finish time after the launch's first instance was taken up, "
                    "solve = the workgroup's time on the instance (device wall clock)"},
        "iterations": {"mean": float(np.mean(iters)), "max": int(np.max(iters))},
        "roofline": {"bound": "hbm", "achieved": nbytes / kernel_s / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": nbytes / kernel_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_batch_solve", "bytes_per_launch": nbytes, "avg_us": kernel_s * 1e6},
        "one_at_a_time": {"value": 1.0 / float(np.mean(one)), "unit": "QPs solved/s",
                          "sample": f"first {len(one)} instances, qp_solve each (FP64, same GPU)"},
        "schedule": sched,
    }
    if not args.no_cpu_baseline:
        import oracle
        nth = oracle.num_threads()
        runs = {}
        for threads, budget in ((nth, 15.0), (1, 10.0)):
            oracle.set_num_threads(threads)
            t = time.perf_counter()
            ns = 0
            while ns < len(qs) and time.perf_counter() - t < budget:
                oracle.solve(qs[ns], tol=args.tol)
                ns += 1
            runs[threads] = (ns, time.perf_counter() - t)
        oracle.set_num_threads(nth)
        ns, el = runs[nth]
        ns1, el1 = runs[1]
        out["cpu_baseline"] = {"value": ns / el, "unit": "QPs solved/s", "cores": nth, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"oracle_qp_solve on the first {ns} instances, one at a time ({el:.1f}s)",
                               "single_thread": {"value": ns1 / el1, "cores": 1,
                                                 "sample": f"the first {ns1} instances ({el1:.1f}s)"}}
    if args.cpu_full:
        out["cpu_full_solve"] = cpu_full("mpc_batch", args.tol, args.cpu_budget_s)
    return out


def portfolio_bytes(q, fam, vb):
    """Algorithmic bytes of one launch of the diagonal-Q path's two products
    (vb = bytes per nonzero: 12 in FP64, 8 with FP32 values and int32
    columns).  rhs: A'y fused with the closed-form primal step, x_bar and the
    Halpern average of x -- the nonzeros, row pointers, y gathered once, x,
    c, q, the x anchor and the box (bound_bytes) read, x_T, x_bar and x
    written.  dual:
    A x_bar fused with the dual step and Halpern on y -- the nonzeros, row
    pointers, x_bar gathered once, y, y anchor, l_c, u_c read, y_T and y
    written."""
    if fam == "rhs":
        return vb * q.nnz_A + 4 * (q.n + 1) + 8 * q.m + 8 * q.n * 7 + bound_bytes(q) * q.n
    return vb * q.nnz_A + 4 * (q.m + 1) + 8 * q.n + 8 * q.m * 6


def main_portfolio(args, torch, P, I):
    t = time.perf_counter()
    q = I.portfolio(0)
    log(f"generated {q.name}: n={q.n} m={q.m} nnz(A)={q.nnz_A} in {time.perf_counter() - t:.1f}s")
    mixed = args.precision == "mixed"
    prec = P.PRECISION_MIXED if mixed else P.PRECISION_FP64
    h = P.qp_create_from(q)
    params = P.qp_params_default(tol=args.tol, timing=args.timing, max_iter=args.max_iter, precision=prec)
    try:
        for w in range(args.warmup):
            st = P.qp_solve_ex(h, params)
            log(f"warmup {w}: {P.STATUS_NAMES[st]}")
        torch.cuda.synchronize()
        lat, infos = [], []
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            a = time.perf_counter()
            st = P.qp_solve_ex(h, params)
            lat.append(time.perf_counter() - a)
            _, x, y, info = P.qp_result(h, q.n, q.m)
            infos.append(info)
            log(f"step {s_}: {P.STATUS_NAMES[st]} {lat[-1] * 1e3:.1f} ms it={info['iterations']}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        # the plain FP64 form on the same GPU, and the result's error against it
        p64 = P.qp_params_default(tol=args.tol, timing=args.timing, max_iter=args.max_iter)
        a = time.perf_counter()
        P.qp_solve_ex(h, p64)
        t64 = time.perf_counter() - a
        _, x64, _, i64 = P.qp_result(h, q.n, q.m)
    finally:
        P.qp_destroy(h)
    solved = all(i["status"] == P.OPTIMAL and max(i["r_primal"], i["r_dual"], i["r_gap"]) <= args.tol
                 for i in infos)
    vb = 8 if mixed else 12
    fams = {}
    for name in ("rhs", "dual"):
        j = P.FAMILIES.index(name)
        tj = sum(i["fam_timed"][j] for i in infos)
        fams[name] = (1e3 * sum(i["fam_ms"][j] for i in infos) / max(tj, 1), tj,
                      infos[-1]["fam_launches"][j])
    dom = max(fams, key=lambda k: fams[k][0] * fams[k][2])
    avg_us = fams[dom][0]
    nbytes = portfolio_bytes(q, dom, vb)
    achieved = nbytes / (avg_us * 1e-6) / 1e9 if fams[dom][1] else None
    f, f64 = infos[-1]["primal_obj"], i64["primal_obj"]
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "QPs solved/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products + f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"factor-model portfolio, {q.n - 1000} assets + 1000 factors, "
                               f"m={q.m}, diagonal Q, tol {args.tol:g}, "
                               f"{'mixed precision' if mixed else 'FP64'}",
                   "n": q.n, "m": q.m, "nnz_A": q.nnz_A, "tol": args.tol},
        "solved": solved,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "iterations": {"outer": infos[-1]["iterations"],
                       "outer_per_s": infos[-1]["iterations"] / np.median(lat)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
                     "kernel": {"rhs": "A'y + closed-form primal step (k_spmv<EpiProx>)",
                                "dual": "A x_bar + dual step + Halpern on y (k_spmv<EpiDual>)"}[dom],
                     "bytes_per_launch": nbytes, "avg_us": avg_us},
        "kernels": {k: {"avg_us": round(v[0], 3), "launches_per_solve": v[2]} for k, v in fams.items()},
        "fp64_plain": {"value": 1.0 / t64, "unit": "QPs solved/s", "iterations": i64["iterations"],
                       "status": P.STATUS_NAMES[i64["status"]]},
        "error_vs_fp64": {"objective_rel": abs(f - f64) / (1 + abs(f64)),
                          "x_inf": float(np.abs(x - x64).max())},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(q, infos[-1], args.cpu_sample_iters or 4096, args.tol)
    if args.cpu_full:
        out["cpu_full_solve"] = cpu_full("portfolio", args.tol, args.cpu_budget_s)
    return out


def main_serve(args, torch, P, I):
    """A Poisson stream of mixed requests through the request server."""
    import threading

    t = time.perf_counter()
    arrivals, qs = I.served_stream(args.requests, rate=args.rate)
    kinds = [q.name.split("_")[0].rstrip("0123456789") for q in qs]
    log(f"generated {len(qs)} requests in {time.perf_counter() - t:.1f}s: "
        + ", ".join(f"{k} {kinds.count(k)}" for k in sorted(set(kinds))))
    mixed = args.precision == "mixed"
    params = P.qp_params_default(tol=args.tol, max_iter=args.max_iter,
                                 precision=P.PRECISION_MIXED if mixed else P.PRECISION_FP64)
    cfg = dict(batch_lanes=args.lanes, general_lanes=args.general_lanes, single_workers=args.workers,
               batch_max_dim=args.batch_max_dim, general_max_dim=args.general_max_dim,
               batch_linger_us=args.linger_us, batch_shape=args.batch_shape, batch_order=args.batch_order)
    with P.Server(params, **cfg) as srv:
        for q in (I.mpc(0), I.random_small(0, n=2000), I.portfolio(0, n_assets=10000, k_factors=50)):
            srv.wait(srv.submit(q))                              # warm-up (not timed)
        ids = [None] * len(qs)
        t0 = time.perf_counter()

        def feed():
            for i, q in enumerate(qs):
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                ids[i] = srv.submit(q)

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        res = []
        for i, rid in enumerate(ids):
            srv.wait(rid)
            res.append(srv.result(rid))
            log(f"request {i + 1}/{len(ids)} ({kinds[i]}, n={qs[i].n}) done at {time.perf_counter() - t0:.1f}s")
        elapsed = time.perf_counter() - t0
    lat = np.array([tm["finished"] - tm["submitted"] for _, tm in res])
    first = min(tm["submitted"] for _, tm in res)
    last = max(tm["finished"] for _, tm in res)
    ok = []
    for q, (g, _) in zip(qs, res):
        bad = q.name.endswith("_infeasible")
        kkt = max(g.info["r_primal"], g.info["r_dual"], g.info["r_gap"])
        ok.append(g.status == P.PRIMAL_INFEASIBLE if bad else (g.status == P.OPTIMAL and kkt <= args.tol))
    per_kind = {}
    for k in sorted(set(kinds)):
        sel = np.array([kk == k for kk in kinds])
        per_kind[k] = {"count": int(sel.sum()), "p50_s": float(np.percentile(lat[sel], 50)),
                       "p99_s": float(np.percentile(lat[sel], 99)),
                       "route": sorted({tm["route"] for (_, tm), s_ in zip(res, sel) if s_})}
    # the plain FP64 form, one solve at a time, on a sample of the same stream
    one, n_one = 0.0, 0
    p64 = P.qp_params_default(tol=args.tol, max_iter=args.max_iter)
    ta = time.perf_counter()
    for q in qs:
        if time.perf_counter() - ta > args.one_at_a_time_s:
            break
        if n_one % 50 == 0:
            log(f"one at a time: {n_one} solved")
        a = time.perf_counter()
        with P.Solver(q) as s1:
            s1.solve(p64)
        one += time.perf_counter() - a
        n_one += 1
    verify = None if args.no_cpu_baseline else verify_served(qs, res, args, P)
    out = {
        "metric": METRIC,
        "value": int(np.sum(ok)) / (last - first),
        "unit": "QPs solved/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products + f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"served stream: {len(qs)} requests, Poisson arrivals at {args.rate:g}/s, "
                               f"60% MPC / 30% random QP n~U(1e3,5e4) / 10% portfolio n~U(1e4,1e5), "
                               f"2% infeasible, tol {args.tol:g}", **cfg,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "solved": int(np.sum(ok)), "requests": len(qs),
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "per_kind": per_kind},
        "roofline": None,
        "one_at_a_time": {"value": n_one / one if one else None, "unit": "QPs solved/s",
                          "sample": f"first {n_one} requests of the stream, qp_create + qp_solve each, FP64"},
        "oracle_verified": verify,
    }
    return out


def verify_served(qs, res, args, P):
    """The served results against the CPU oracle: a seeded 5 % sample of the
    requests plus every infeasible one, smallest first, within
    --verify-budget-s of oracle time.  A result is verified when its status
    is the oracle's and, if OPTIMAL, the oracle's KKT evaluation of the
    returned point is <= tol and the objective is within 1e-6 (1 + |f|) of
    the oracle's (solved at tol 1e-9, or 1e-7 above 20,000 variables)."""
    import oracle
    rng = np.random.default_rng(SERVE_VERIFY_SEED)
    pick = set(int(i) for i in rng.choice(len(qs), size=max(1, int(round(0.05 * len(qs)))), replace=False))
    pick |= {i for i, q in enumerate(qs) if q.name.endswith("_infeasible")}
    order = sorted(pick, key=lambda i: qs[i].n + qs[i].m)
    t0 = time.perf_counter()
    rows, by_kind = [], {}
    for i in order:
        if time.perf_counter() - t0 > args.verify_budget_s:
            break
        q, (g, _) = qs[i], res[i]
        ref_tol = 1e-9 if q.n <= 20000 else 1e-7
        o = oracle.solve(q, tol=ref_tol, max_iter=1_000_000)
        good = g.status == o.status
        kkt = ferr = None
        if good and o.status == P.OPTIMAL:
            k = oracle.kkt(q, g.x, g.y)
            kkt = max(k["r_primal"], k["r_dual"], k["r_gap"])
            ferr = abs(g.info["primal_obj"] - o.info["primal_obj"]) / (1 + abs(o.info["primal_obj"]))
            good = kkt <= args.tol and ferr <= 1e-6
        kind = q.name.split("_")[0].rstrip("0123456789")
        b = by_kind.setdefault(kind, [0, 0])
        b[0] += 1
        b[1] += int(good)
        rows.append({"request": i, "name": q.name, "n": q.n, "status": P.STATUS_NAMES[g.status],
                     "oracle_status": oracle.STATUS_NAMES[o.status], "kkt": kkt, "objective_rel_err": ferr,
                     "verified": bool(good)})
        log(f"verify request {i} ({q.name}): {rows[-1]['status']} vs oracle {rows[-1]['oracle_status']}, "
            f"kkt {kkt}, objective error {ferr}: {'ok' if good else 'MISMATCH'}")
    oracle_s = time.perf_counter() - t0
    # the same checked requests solved again by the oracle on one thread
    # (standalone serve runs; the default line skips it)
    single = None
    if getattr(args, "verify_single_thread", False) and rows:
        nth = oracle.num_threads()
        oracle.set_num_threads(1)
        t1, done = time.perf_counter(), 0
        try:
            for r in rows:
                if time.perf_counter() - t1 > args.verify_budget_s:
                    break
                q = qs[r["request"]]
                oracle.solve(q, tol=1e-9 if q.n <= 20000 else 1e-7, max_iter=1_000_000)
                done += 1
        finally:
            oracle.set_num_threads(nth)
        el1 = time.perf_counter() - t1
        single = {"requests": done, "seconds": el1, "cores": 1,
                  "note": f"the first {done} checked requests again on one thread (the 16-thread pass above "
                          f"took {oracle_s:.1f} s for all {len(rows)})"}
    return {"selected": len(order), "checked": len(rows), "verified": sum(r["verified"] for r in rows),
            "by_kind": {k: {"checked": v[0], "verified": v[1]} for k, v in by_kind.items()},
            "oracle_seconds": oracle_s, "cores": oracle.num_threads(), "single_thread": single,
            "sample": f"seeded 5% of {len(qs)} requests (seed {SERVE_VERIFY_SEED}) plus every infeasible request, "
                      f"smallest first, {args.verify_budget_s:g}s oracle budget",
            "mismatches": [r for r in rows if not r["verified"]]}


def parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--timing", type=int, default=64,
                    help="time every k-th launch per kernel family with HIP events (each timed launch "
                         "costs about 7 us of event records; 64 keeps that near 0.5%% of a solve)")
    ap.add_argument("--lag", type=int, default=1, help="inner steps queued ahead of the host's view")
    ap.add_argument("--max-iter", type=int, default=100000,
                    help="outer iteration cap (lower only for short profiling runs)")
    ap.add_argument("--workload", choices=["large_sparse", "small", "mpc_batch", "portfolio", "serve"],
                    default="large_sparse")
    ap.add_argument("--requests", type=int, default=200, help="requests of the served stream")
    ap.add_argument("--rate", type=float, default=2000.0, help="arrivals per second of the served stream")
    ap.add_argument("--lanes", type=int, default=2, help="server lanes for diagonal-Q requests")
    ap.add_argument("--general-lanes", type=int, default=2, help="server lanes for non-diagonal-Q requests")
    ap.add_argument("--workers", type=int, default=5, help="server single-path workers")
    ap.add_argument("--batch-max-dim", type=int, default=20000)
    ap.add_argument("--general-max-dim", type=int, default=3000)
    ap.add_argument("--linger-us", type=float, default=200.0)
    ap.add_argument("--one-at-a-time-s", type=float, default=20.0,
                    help="seconds spent solving the served stream one request at a time (FP64)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="arithmetic of the portfolio and batched workloads (default: mixed for them; "
                         "the large sparse workload is FP64)")
    ap.add_argument("--count", type=int, default=4096, help="instances of the batched workload")
    ap.add_argument("--schedule", default="auto",
                    help="batched launch schedule: auto (autotuner), default, or SHAPE,ORDER")
    ap.add_argument("--batch-shape", type=int, default=-1, help="server batched launch shape (-1: default)")
    ap.add_argument("--batch-order", type=int, default=-1, help="server batched queue order (-1: default)")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="served stream: HIP hardware queues of the process (GPU_MAX_HW_QUEUES, set before "
                         "the first HIP call when not already set; 0 keeps the runtime's default of 4, "
                         "which measured faster than 16 on the served stream); at most 32")
    ap.add_argument("--one-at-a-time", type=int, default=32,
                    help="instances of the batched workload also solved one by one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 64 MiB (scale for rocprofv3 byte counters)")
    ap.add_argument("--cpu-sample-iters", type=int, default=None,
                    help="outer iterations of the oracle's timed sample (default: per workload)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle's whole solve (child process, --cpu-budget-s)")
    ap.add_argument("--cpu-budget-s", type=float, default=900.0)
    ap.add_argument("--oracle-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-secondary", action="store_true",
                    help="default workload only: skip the other workloads' figures")
    ap.add_argument("--verify-budget-s", type=float, default=90.0,
                    help="oracle time for verifying the served stream's sample")
    ap.add_argument("--no-verify-single-thread", dest="verify_single_thread", action="store_false",
                    help="serve: skip timing the verified sample again on one oracle thread")
    return ap


def main():
    args = parser().parse_args()

    if args.oracle_child:
        return oracle_child(args.oracle_child, args.tol)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve" and args.hw_queues > 0 and "GPU_MAX_HW_QUEUES" not in os.environ:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))

    import torch

    if args.copy_calibration:
        src = torch.zeros(8 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 copies of 67108864 bytes each way")
        return

    import paper_2602_23967_amd as P
    from paper_2602_23967_amd import instances as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "mpc_batch":
        if args.precision is None:
            args.precision = "mixed"
        print(json.dumps(main_batch(args, torch, P, I)), flush=True)
        return
    if args.workload == "portfolio":
        if args.precision is None:
            args.precision = "mixed"
        print(json.dumps(main_portfolio(args, torch, P, I)), flush=True)
        return
    if args.workload == "serve":
        if args.precision is None:
            args.precision = "mixed"
        out = main_serve(args, torch, P, I)
    else:
        out = main_single(args, torch, P, I)
        if args.workload == "large_sparse" and not args.no_secondary:
            out["secondary"] = run_secondary(args, torch, P, I)
    print(json.dumps(out), flush=True)


def main_single(args, torch, P, I):
    """One problem through qp_create / qp_solve: the n = 1e6 QP (default)
    or the n = 1000 QP (--workload small)."""
    t = time.perf_counter()
    small = args.workload == "small"
    q = I.random_small(0) if small else I.large_sparse(0, n=args.n)
    log(f"generated {q.name}: n={q.n} m={q.m} nnz(Q)={q.nnz_Q} nnz(A)={q.nnz_A} "
        f"in {time.perf_counter() - t:.1f}s")
    h = P.qp_create_from(q)
    params = P.qp_params_default(tol=args.tol, timing=args.timing, inner_lag=args.lag,
                                 max_iter=args.max_iter)
    try:
        for w in range(args.warmup):
            st = P.qp_solve_ex(h, params)
            log(f"warmup {w}: {P.STATUS_NAMES[st]}")
        torch.cuda.synchronize()
        lat, infos = [], []
        t_start = time.perf_counter()
        for s in range(args.steps):
            a = time.perf_counter()
            st = P.qp_solve_ex(h, params)
            lat.append(time.perf_counter() - a)
            _, x, y, info = P.qp_result(h, q.n, q.m)
            infos.append(info)
            log(f"step {s}: {P.STATUS_NAMES[st]} {lat[-1]:.3f}s it={info['iterations']} "
                f"inner={info['inner_iterations']} kkt=({info['r_primal']:.1e},{info['r_dual']:.1e},"
                f"{info['r_gap']:.1e})")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
    finally:
        _, x, y, info = P.qp_result(h, q.n, q.m)
        P.qp_destroy(h)

    solved = all(i["status"] == P.OPTIMAL and max(i["r_primal"], i["r_dual"], i["r_gap"]) <= args.tol
                 for i in infos)
    # the dominant kernel: the fused inner H p product
    f = P.FAMILIES.index("spmv_hp")
    timed = sum(i["fam_timed"][f] for i in infos)
    ms = sum(i["fam_ms"][f] for i in infos)
    avg_us = 1e3 * ms / max(timed, 1)
    nbytes = hp_bytes(q.n, q.nnz_Q, bound_bytes(q))
    # launches that found the inner solve already stopped return at once; their
    # time stays in the denominator, their bytes do not count
    launches = sum(i["fam_launches"][f] for i in infos)
    active = sum(i["spmv_hp_active"] for i in infos)
    achieved = nbytes * active / (avg_us * 1e-6 * launches) / 1e9 if timed else None
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernels_digest") == kernels_digest():
            traffic = tr.get("bytes_per_launch")
    kern = {}
    for j, name in enumerate(P.FAMILIES):
        tj = sum(i["fam_timed"][j] for i in infos)
        if tj:
            kern[name] = {"avg_us": round(1e3 * sum(i["fam_ms"][j] for i in infos) / tj, 3),
                          "launches_per_solve": infos[-1]["fam_launches"][j]}
    # the product's random gathers (one per nonzero) against the device's
    # measured gather rate for the same vector length and part keying: the
    # bound this product actually meets (outside the timed region)
    gather = None
    if timed:
        peak_g = P.measure_gather_rate(q.n, q.nnz_Q, 20)
        ach_g = q.nnz_Q * active / (avg_us * 1e-6 * launches)
        gather = {"achieved": ach_g / 1e9, "peak": peak_g / 1e9, "unit": "G gathers/s",
                  "frac": ach_g / peak_g if peak_g > 0 else None,
                  "peak_source": "qp_measure_gather_rate (random 8-byte gathers, XCD-keyed parts, "
                                 f"n={q.n}, {q.nnz_Q} per launch)"}
        log(f"gather rate: product {ach_g / 1e9:.0f} G/s, device {peak_g / 1e9:.0f} G/s")

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "QPs solved/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"tiny random convex QP n={q.n} m={q.m} (half '=', half '>='), "
                                f"Q = B'B + 0.01 I, A at 1%, box [-1,1], tol {args.tol:g}") if small else
                               (f"large sparse convex QP n={q.n} m={q.m} (half '=', half '>='), "
                                f"Q SPD ~10 off-diagonals/row, A 8 nnz/row, box [0,10], tol {args.tol:g}"),
                   "n": q.n, "m": q.m, "nnz_Q": q.nnz_Q, "nnz_A": q.nnz_A, "tol": args.tol},
        "solved": solved,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "iterations": {"outer": infos[-1]["iterations"], "inner": infos[-1]["inner_iterations"],
                       "outer_per_s": infos[-1]["iterations"] / np.median(lat),
                       "inner_per_s": infos[-1]["inner_iterations"] / np.median(lat)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                     "kernel": ("inner H p product (k_spmv<EpiStepA>)" if small else
                                "inner H p product (k_spmv<EpiStepA> + k_rows<EpiStepA>)"),
                     "bytes_per_launch": nbytes, "avg_us": avg_us, "timed_launches": timed,
                     "launches": launches, "active_launches": active},
        "gather_roofline": gather,
        "kernels": kern,
        "setup_s": info["setup_seconds"],
        # the problem handed over in host memory: qp_create (upload, host
        # preparation, norm estimates) plus one solve with its result download
        "pcie_inclusive": {"value": 1.0 / (info["setup_seconds"] + elapsed / args.steps),
                           "unit": "QPs solved/s",
                           "note": "qp_create from host arrays + qp_solve + qp_result, one problem"},
    }
    if small:
        # launch-bound: the latency of one iteration is the figure that matters
        med = float(np.median(lat))
        fam_us = {k: v["avg_us"] for k, v in kern.items()}
        out["latency_us"] = {
            "per_outer_iteration": 1e6 * med / max(infos[-1]["iterations"], 1),
            "per_inner_step_kernels": sum(fam_us.get(k, 0.0) for k in ("dir", "spmv_hp", "update")),
            "note": ("per_outer_iteration = solve wall time / outer iterations (inner steps included); "
                     "per_inner_step_kernels = event-timed main kernels of one inner step (direction, H p, "
                     "update; finishing kernels and launch gaps not included)")}
    if not args.no_cpu_baseline:
        if small:
            out["cpu_baseline"] = cpu_small(q, args.tol)
        else:
            out["cpu_baseline"] = cpu_baseline(q, infos[-1], args.cpu_sample_iters or 24, args.tol)
            full = measured_full_solve("large_sparse", args.tol)
            if full is not None:
                out["cpu_baseline"]["full_solve_measured"] = full
    if args.cpu_full and not small:
        out["cpu_full_solve"] = cpu_full("large_sparse", args.tol, args.cpu_budget_s)
        log(f"oracle full solve: {out['cpu_full_solve']}")
    return out


def summary(out):
    """The figures of a workload's line that the default run attaches for
    the other workloads (measured in the same run)."""
    keep = ("value", "unit", "ms_per_step", "steps", "dtype", "solved", "solved_count", "requests", "iterations",
            "latency_s", "latency_us", "fp64_plain", "one_at_a_time", "error_vs_fp64", "oracle_verified",
            "instance_times_ms")
    d = {k: out[k] for k in keep if k in out}
    d["workload"] = out["config"]["workload"]
    r = out.get("roofline")
    if r:
        d["roofline"] = {k: r.get(k) for k in ("bound", "achieved", "peak", "unit", "frac", "kernel", "avg_us")}
    return d


def run_secondary(args, torch, P, I):
    """The other workloads' lines in the default run: the factor portfolio
    (mixed precision, with its FP64 solve), the 4096-instance MPC batch
    (mixed, autotuned), the n = 1000 QP (FP64, launch-bound) and the served
    stream (mixed), each timed as its own --workload run would be, without
    CPU baselines; the served stream keeps its oracle check of a sample
    (unless --no-cpu-baseline) with shorter budgets for that check and for
    its one-at-a-time comparison."""
    import copy
    res = {}
    runs = {"portfolio": main_portfolio, "mpc_batch": main_batch, "small": main_single, "serve": main_serve}
    for wl, prec, steps in (("portfolio", "mixed", 3), ("mpc_batch", "mixed", 3), ("small", None, 5),
                            ("serve", "mixed", 1)):
        a = copy.copy(args)
        a.workload, a.precision, a.steps, a.warmup = wl, prec, steps, 1
        a.no_cpu_baseline, a.cpu_full = True, False
        if wl == "serve":
            a.no_cpu_baseline = args.no_cpu_baseline
            a.verify_budget_s = min(args.verify_budget_s, 45.0)
            a.one_at_a_time_s = min(args.one_at_a_time_s, 15.0)
            a.verify_single_thread = False
        t = time.perf_counter()
        out = runs[wl](a, torch, P, I)
        res[wl] = summary(out)
        log(f"secondary {wl}: {res[wl]['value']:.4g} {res[wl]['unit']} ({time.perf_counter() - t:.0f}s)")
    return res


if __name__ == "__main__":
    main()
