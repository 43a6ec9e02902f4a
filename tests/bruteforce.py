"""Exact references for tiny problems, written from first principles and
independent of the oracle and of the HIP path.

* ``box_qp_enum``: minimiser of 1/2 x'Hx - r'x over a box by enumerating every
  assignment of {at lower, at upper, free} to the coordinates and keeping the
  one whose stationary point satisfies the sign conditions (H positive
  definite, so exactly one does).
* ``qp_enum``: minimiser of a tiny QP by enumerating active sets of bounds
  and rows; every candidate is the solution of an equality-constrained QP,
  and the feasible candidate with the least objective is the optimum.
"""

from __future__ import annotations

import itertools

import numpy as np


def box_qp_enum(H, r, l, u, tol=1e-10):
    n = H.shape[0]
    states = []
    for i in range(n):
        s = ["F"]
        if np.isfinite(l[i]):
            s.append("L")
        if np.isfinite(u[i]) and u[i] > l[i]:
            s.append("U")
        if l[i] == u[i]:
            s = ["L"]
        states.append(s)
    best = None
    for combo in itertools.product(*states):
        x = np.zeros(n)
        F = [i for i in range(n) if combo[i] == "F"]
        for i in range(n):
            if combo[i] == "L":
                x[i] = l[i]
            elif combo[i] == "U":
                x[i] = u[i]
        if F:
            Fx = np.array(F)
            fixed = np.array([i for i in range(n) if combo[i] != "F"], dtype=int)
            rhs = r[Fx] - (H[np.ix_(Fx, fixed)] @ x[fixed] if fixed.size else 0.0)
            x[Fx] = np.linalg.solve(H[np.ix_(Fx, Fx)], rhs)
        if np.any(x < l - tol) or np.any(x > u + tol):
            continue
        g = H @ x - r
        ok = True
        for i in range(n):
            if combo[i] == "F" and abs(g[i]) > 1e-8 * (1 + np.abs(r).max()):
                ok = False
            if combo[i] == "L" and l[i] < u[i] and g[i] < -tol:
                ok = False
            if combo[i] == "U" and g[i] > tol:
                ok = False
        if ok:
            f = 0.5 * x @ H @ x - r @ x
            if best is None or f < best[1]:
                best = (x, f)
    assert best is not None
    return best[0]


def qp_enum(Q, c, A, lc, uc, lv, uv, feas_tol=1e-9):
    """Returns (x*, f*) of min 1/2 x'Qx + c'x, lc <= Ax <= uc, lv <= x <= uv."""
    Q = np.asarray(Q, float)
    A = np.asarray(A, float)
    n, m = Q.shape[0], A.shape[0]
    vstates = []
    for i in range(n):
        if lv[i] == uv[i]:
            vstates.append(["L"])
            continue
        s = ["F"]
        if np.isfinite(lv[i]):
            s.append("L")
        if np.isfinite(uv[i]):
            s.append("U")
        vstates.append(s)
    rstates = []
    for j in range(m):
        if lc[j] == uc[j]:
            rstates.append(["lo"])
            continue
        s = ["off"]
        if np.isfinite(lc[j]):
            s.append("lo")
        if np.isfinite(uc[j]):
            s.append("hi")
        rstates.append(s)
    best = None
    for vc in itertools.product(*vstates):
        fixed = [i for i in range(n) if vc[i] != "F"]
        free = [i for i in range(n) if vc[i] == "F"]
        xf = np.array([lv[i] if vc[i] == "L" else uv[i] for i in fixed])
        for rc in itertools.product(*rstates):
            act = [j for j in range(m) if rc[j] != "off"]
            bnd = np.array([lc[j] if rc[j] == "lo" else uc[j] for j in act])
            x = np.zeros(n)
            x[fixed] = xf
            if free:
                Fi = np.array(free)
                Fx = np.array(fixed, dtype=int)
                qf = Q[np.ix_(Fi, Fi)]
                rhs1 = -c[Fi] - (Q[np.ix_(Fi, Fx)] @ xf if Fx.size else 0.0)
                if act:
                    Aa = A[np.ix_(act, Fi)]
                    rhs2 = bnd - (A[np.ix_(act, Fx)] @ xf if Fx.size else 0.0)
                    K = np.block([[qf, Aa.T], [Aa, np.zeros((len(act), len(act)))]])
                    rhs = np.concatenate([rhs1, rhs2])
                else:
                    K, rhs = qf, rhs1
                sol, *_ = np.linalg.lstsq(K, rhs, rcond=None)
                if np.linalg.norm(K @ sol - rhs) > 1e-9 * (1 + np.linalg.norm(rhs)):
                    continue
                x[Fi] = sol[: len(free)]
            else:
                if act and np.abs(A[act] @ x - bnd).max() > feas_tol:
                    continue
            ax = A @ x
            if np.any(x < lv - feas_tol) or np.any(x > uv + feas_tol):
                continue
            if np.any(ax < lc - feas_tol) or np.any(ax > uc + feas_tol):
                continue
            f = 0.5 * x @ Q @ x + c @ x
            if best is None or f < best[1] - 1e-14:
                best = (x, f)
    assert best is not None, "no feasible active set"
    return best


def lc_uc(b, sense):
    """Row bounds from right-hand sides and senses, written for the tests."""
    lc = np.array([b[i] if s in (ord("E"), ord("G")) else -np.inf for i, s in enumerate(sense)])
    uc = np.array([b[i] if s in (ord("E"), ord("L")) else np.inf for i, s in enumerate(sense)])
    return lc, uc
