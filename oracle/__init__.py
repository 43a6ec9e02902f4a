"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The product library never does.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

NOT_SOLVED, OPTIMAL, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, ITERATION_LIMIT, NUMERICAL_ERROR = range(6)
STATUS_NAMES = {0: "NOT_SOLVED", 1: "OPTIMAL", 2: "PRIMAL_INFEASIBLE", 3: "DUAL_INFEASIBLE",
                4: "ITERATION_LIMIT", 5: "NUMERICAL_ERROR"}
INNER_AUTO, INNER_MPRGP, INNER_BB, INNER_CLOSED = range(4)

_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
_lp = C.POINTER(C.c_int64)
_ip = C.POINTER(C.c_int32)


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", _i64), ("check_every", _i64),
                ("max_inner", _i64), ("inner_solver", C.c_int), ("use_halpern", C.c_int),
                ("theta", C.c_double), ("kp", C.c_double), ("ki", C.c_double), ("kd", C.c_double),
                ("gamma_inner", C.c_double), ("eps_min", C.c_double),
                ("eps_inner_fixed", C.c_double), ("restart_sufficient", C.c_double),
                ("restart_necessary", C.c_double), ("restart_artificial", C.c_double),
                ("eps_inf", C.c_double), ("eta_scale", C.c_double), ("norm_safety", C.c_double),
                ("power_tol", C.c_double), ("power_max_iter", _i64), ("mprgp_gamma", C.c_double),
                ("mprgp_abar_scale", C.c_double), ("verbose", C.c_int)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", _i64), ("inner_iterations", _i64),
                ("restarts", _i64), ("checks", _i64), ("r_primal", C.c_double),
                ("r_dual", C.c_double), ("r_gap", C.c_double), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("omega", C.c_double), ("eta", C.c_double),
                ("norm_A", C.c_double), ("norm_Q", C.c_double), ("eps_inner", C.c_double),
                ("natural_residual", C.c_double), ("seconds_setup", C.c_double),
                ("seconds_inner", C.c_double), ("seconds_check", C.c_double),
                ("seconds_total", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.oracle_params_default.argtypes = [C.POINTER(Params)]
        L.oracle_bounds_from_sense.argtypes = [_i64, _dp, C.c_char_p, _dp, _dp]
        L.oracle_qp_solve.argtypes = [_i64, _i64, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp, _dp,
                                      _dp, _dp, C.POINTER(Params), _dp, _dp, C.POINTER(Info)]
        L.oracle_kkt.argtypes = [_i64, _i64, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp, _dp, _dp,
                                 _dp, _dp, _dp, _dp]
        L.oracle_subproblem.argtypes = [_i64, _lp, _ip, _dp, _dp, _dp, C.c_double, _dp, _dp,
                                        C.c_double, _i64, C.c_int, C.c_double, _dp]
        L.oracle_subproblem.restype = _i64
        L.oracle_norm2.argtypes = [_i64, _i64, _lp, _ip, _dp, C.c_double, _i64, _lp]
        L.oracle_norm2.restype = C.c_double
        L.oracle_csr_matvec.argtypes = [_i64, _lp, _ip, _dp, _dp, _dp]
        L.oracle_support.argtypes = [_i64, _dp, _dp, _dp]
        L.oracle_support.restype = C.c_double
        L.oracle_primal_infeasible.argtypes = [_i64, _i64, _lp, _ip, _dp, _dp, _dp, _dp, _dp,
                                               _dp, C.c_double, _dp]
        L.oracle_dual_infeasible.argtypes = [_i64, _i64, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp,
                                             _dp, _dp, _dp, _dp, C.c_double, C.c_double, _dp]
        L.oracle_splitmix_unit.argtypes = [C.c_uint64]
        L.oracle_splitmix_unit.restype = C.c_double
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        L.oracle_set_num_threads.restype = None
        L.oracle_halpern.argtypes = [_i64, _i64, C.c_double, _dp, _dp, _dp, _dp]
        L.oracle_pid.argtypes = [C.c_double] * 7 + [_dp, _dp]
        L.oracle_pid.restype = C.c_double
        L.oracle_inner_tol.argtypes = [C.c_double] * 6
        L.oracle_inner_tol.restype = C.c_double
        L.oracle_restart_test.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, _i64,
                                          _i64, C.POINTER(Params)]
        _lib = L
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _csr(M):
    if M is None:
        return None, None, None, ()
    M = M.tocsr()
    M.sum_duplicates()
    M.sort_indices()
    p = np.ascontiguousarray(M.indptr, dtype=np.int64)
    j = np.ascontiguousarray(M.indices, dtype=np.int32)
    v = np.ascontiguousarray(M.data, dtype=np.float64)
    return p.ctypes.data_as(_lp), j.ctypes.data_as(_ip), v.ctypes.data_as(_dp), (p, j, v)


def params(**kw) -> Params:
    p = Params()
    lib().oracle_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def bounds_from_sense(b, sense: bytes):
    b = _f64(b)
    m = b.shape[0]
    lc = np.empty(m)
    uc = np.empty(m)
    if lib().oracle_bounds_from_sense(m, _d(b), sense, _d(lc), _d(uc)) != 0:
        raise ValueError("unknown sense")
    return lc, uc


@dataclass
class Result:
    status: int
    x: np.ndarray
    y: np.ndarray
    info: dict

    @property
    def status_name(self):
        return STATUS_NAMES[self.status]


def solve(qp, prm: Params | None = None, **kw) -> Result:
    """Solve a paper_2602_23967_amd.instances.QP with the oracle."""
    prm = prm if prm is not None else params(**kw)
    lc, uc = bounds_from_sense(qp.b, qp.sense)
    qp_, qj_, qv_, keepq = _csr(qp.Q)
    ap_, aj_, av_, keepa = _csr(qp.A)
    c, lv, uv = _f64(qp.c), _f64(qp.lb), _f64(qp.ub)
    x = np.zeros(qp.n)
    y = np.zeros(max(qp.m, 1))
    info = Info()
    st = lib().oracle_qp_solve(qp.n, qp.m, qp_, qj_, qv_, ap_, aj_, av_, _d(c), _d(lc), _d(uc),
                               _d(lv), _d(uv), C.byref(prm), _d(x), _d(y), C.byref(info))
    if st < 0:
        raise ValueError("oracle_qp_solve rejected the input")
    return Result(st, x, y[: qp.m], info.as_dict())


def kkt(qp, x, y):
    """dict of r_primal, r_dual, r_gap, pobj, dobj, natural, pviol at (x, y)."""
    lc, uc = bounds_from_sense(qp.b, qp.sense)
    qp_, qj_, qv_, keepq = _csr(qp.Q)
    ap_, aj_, av_, keepa = _csr(qp.A)
    c, lv, uv = _f64(qp.c), _f64(qp.lb), _f64(qp.ub)
    x = _f64(x)
    y = _f64(y) if qp.m > 0 else np.zeros(1)
    out = np.zeros(7)
    lib().oracle_kkt(qp.n, qp.m, qp_, qj_, qv_, ap_, aj_, av_, _d(c), _d(lc), _d(uc), _d(lv),
                     _d(uv), _d(x), _d(y), _d(out))
    return dict(zip(["r_primal", "r_dual", "r_gap", "pobj", "dobj", "natural", "pviol"], out))


def subproblem(Q, lv, uv, tau, rhs, x0, eps, max_inner=10000, solver=INNER_AUTO, norm_Q=None):
    """argmin over [lv, uv] of 1/2 x'(Q + I/tau)x - rhs'x from warm start x0.
    Returns (x, iterations, final projected-gradient norm)."""
    n = rhs.shape[0]
    if norm_Q is None:
        norm_Q = 0.0 if Q is None else 1.01 * norm2(Q)
    qp_, qj_, qv_, keep = _csr(Q)
    lv, uv, rhs = _f64(lv), _f64(uv), _f64(rhs)
    x = np.array(x0, dtype=np.float64, copy=True)
    res = C.c_double(0.0)
    it = lib().oracle_subproblem(n, qp_, qj_, qv_, _d(lv), _d(uv), float(tau), _d(rhs), _d(x),
                                 float(eps), int(max_inner), int(solver), float(norm_Q),
                                 C.byref(res))
    if it < 0:
        raise ValueError("closed form requested for a non-diagonal Q")
    return x, int(it), res.value


def norm2(M, tol=1e-7, max_iter=1000):
    p_, j_, v_, keep = _csr(M)
    its = C.c_int64(0)
    r, c = M.shape
    return lib().oracle_norm2(r, c, p_, j_, v_, tol, max_iter, C.byref(its))


def matvec(M, x):
    p_, j_, v_, keep = _csr(M)
    x = _f64(x)
    y = np.zeros(M.shape[0])
    lib().oracle_csr_matvec(M.shape[0], p_, j_, v_, _d(x), _d(y))
    return y


def support(z, l, u):
    z, l, u = _f64(z), _f64(l), _f64(u)
    return lib().oracle_support(z.shape[0], _d(z), _d(l), _d(u))


def primal_infeasible(qp, dy, eps_inf=1e-8):
    lc, uc = bounds_from_sense(qp.b, qp.sense)
    ap_, aj_, av_, keep = _csr(qp.A)
    lv, uv, dy = _f64(qp.lb), _f64(qp.ub), _f64(dy)
    ray = np.zeros(qp.m)
    f = lib().oracle_primal_infeasible(qp.n, qp.m, ap_, aj_, av_, _d(lc), _d(uc), _d(lv),
                                       _d(uv), _d(dy), eps_inf, _d(ray))
    return bool(f), ray


def dual_infeasible(qp, dx, eps_tol=1e-6, eps_inf=1e-8):
    lc, uc = bounds_from_sense(qp.b, qp.sense)
    qp_, qj_, qv_, keepq = _csr(qp.Q)
    ap_, aj_, av_, keepa = _csr(qp.A)
    c, lv, uv, dx = _f64(qp.c), _f64(qp.lb), _f64(qp.ub), _f64(dx)
    ray = np.zeros(qp.n)
    f = lib().oracle_dual_infeasible(qp.n, qp.m, qp_, qj_, qv_, ap_, aj_, av_, _d(c), _d(lc),
                                     _d(uc), _d(lv), _d(uv), _d(dx), eps_tol, eps_inf, _d(ray))
    return bool(f), ray


def splitmix_unit(i: int) -> float:
    return lib().oracle_splitmix_unit(i)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def halpern(t, theta, zt, z, za):
    zt, z, za = _f64(zt), _f64(z), _f64(za)
    out = np.zeros_like(zt)
    lib().oracle_halpern(zt.shape[0], int(t), float(theta), _d(zt), _d(z), _d(za), _d(out))
    return out


def pid(omega, omega0, mx, my, kp, ki, kd, integral=0.0, prev_e=0.0):
    """Returns (new omega, integral, prev_e)."""
    I_ = C.c_double(integral)
    P_ = C.c_double(prev_e)
    w = lib().oracle_pid(omega, omega0, mx, my, kp, ki, kd, C.byref(I_), C.byref(P_))
    return w, I_.value, P_.value


def inner_tol(eps_prev, gamma, omega, tau, move, eps_min):
    return lib().oracle_inner_tol(eps_prev, gamma, omega, tau, move, eps_min)


def restart_test(R, R_start, R_prev, R_prev_valid, t, k, prm: Params | None = None):
    prm = prm if prm is not None else params()
    return bool(lib().oracle_restart_test(R, R_start, R_prev, int(R_prev_valid), int(t), int(k),
                                          C.byref(prm)))
