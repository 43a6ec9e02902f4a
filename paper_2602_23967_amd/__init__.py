"""Python binding of libpdhcg_hip.so, the gfx950 PDHCG-II convex-QP solver.

The functions mirror the C ABI of include/pdhcg.h one to one and only
marshal arguments: every step of the method runs in the library's HIP
kernels.  Device buffers for the operator-level calls are torch tensors on
the GPU (float64); torch provides device memory and streams only.

The library is loaded from this package directory; if it is missing the
import of the binding functions raises (there is no CPU fallback).
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdhcg_hip.so")

NOT_SOLVED, OPTIMAL, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, ITERATION_LIMIT, NUMERICAL_ERROR = range(6)
STATUS_NAMES = {0: "NOT_SOLVED", 1: "OPTIMAL", 2: "PRIMAL_INFEASIBLE", 3: "DUAL_INFEASIBLE",
                4: "ITERATION_LIMIT", 5: "NUMERICAL_ERROR"}
ERR_INVALID_ARG, ERR_NOT_SYMMETRIC, ERR_DEVICE, ERR_STATE = -1, -2, -3, -4
OP_Q, OP_A, OP_AT = 0, 1, 2
PRECISION_FP64, PRECISION_MIXED = 0, 1
FAMILIES = ["spmv_hp", "update", "dir", "rhs", "ginit", "dual", "halpx", "check"]
NFAM = len(FAMILIES)

_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
_lp = C.POINTER(C.c_int64)
_ip = C.POINTER(C.c_int32)


class QPParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", _i64), ("check_every", _i64),
                ("max_inner", _i64), ("use_halpern", C.c_int), ("inner_lag", C.c_int),
                ("theta", C.c_double), ("kp", C.c_double), ("ki", C.c_double), ("kd", C.c_double),
                ("gamma_inner", C.c_double), ("eps_min", C.c_double),
                ("eps_inner_fixed", C.c_double), ("restart_sufficient", C.c_double),
                ("restart_necessary", C.c_double), ("restart_artificial", C.c_double),
                ("eps_inf", C.c_double), ("eta_scale", C.c_double), ("norm_safety", C.c_double),
                ("power_tol", C.c_double), ("power_max_iter", _i64),
                ("mprgp_gamma", C.c_double), ("mprgp_abar_scale", C.c_double),
                ("timing", C.c_int), ("precision", C.c_int), ("graph_steps", C.c_int),
                ("reserved", C.c_int)]


class QPInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("precision", C.c_int), ("iterations", _i64),
                ("inner_iterations", _i64), ("restarts", _i64), ("checks", _i64),
                ("r_primal", C.c_double), ("r_dual", C.c_double), ("r_gap", C.c_double),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("natural_residual", C.c_double), ("omega", C.c_double), ("eta", C.c_double),
                ("norm_A", C.c_double), ("norm_Q", C.c_double), ("eps_inner", C.c_double),
                ("solve_seconds", C.c_double), ("setup_seconds", C.c_double),
                ("fam_ms", C.c_double * NFAM), ("fam_timed", _i64 * NFAM),
                ("fam_launches", _i64 * NFAM), ("spmv_hp_active", _i64)]

    def as_dict(self):
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v) if f.startswith("fam_") else v
        return d


class ServerConfig(C.Structure):
    _fields_ = [("device_budget", _i64), ("batch_max_dim", _i64), ("general_max_dim", _i64),
                ("batch_lanes", C.c_int32), ("general_lanes", C.c_int32),
                ("single_workers", C.c_int32), ("max_batch", C.c_int32),
                ("batch_shape", C.c_int32), ("batch_order", C.c_int32),
                ("general_shape", C.c_int32), ("diag_workers", C.c_int32),
                ("batch_linger_us", C.c_double)]


class RequestTimes(C.Structure):
    _fields_ = [("submitted", C.c_double), ("started", C.c_double), ("finished", C.c_double),
                ("route", C.c_int32), ("batch_size", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class QPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(the HIP library is required; there is no fallback)")
        L = C.CDLL(LIB_PATH)
        L.qp_params_default.restype = QPParams
        L.qp_create.argtypes = [_i64, _i64, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp, C.c_char_p,
                                _dp, _dp, C.POINTER(C.c_void_p)]
        L.qp_create_ranged.argtypes = [_i64, _i64, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp, _dp,
                                       _dp, _dp, C.POINTER(C.c_void_p)]
        L.qp_create_factored.argtypes = [_i64, _i64, _lp, _ip, _dp, _i64, _lp, _ip, _dp, _lp, _ip, _dp,
                                         _dp, _dp, C.c_char_p, _dp, _dp, C.POINTER(C.c_void_p)]
        L.qp_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.qp_solve.argtypes = [C.c_void_p, C.c_double, _i64]
        L.qp_solve_ex.argtypes = [C.c_void_p, C.POINTER(QPParams)]
        L.qp_result.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(QPInfo)]
        L.qp_destroy.argtypes = [C.c_void_p]
        L.qp_destroy.restype = None
        L.qp_last_error.restype = C.c_char_p
        L.qp_apply.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.qp_dot.argtypes = [C.c_void_p, _i64, C.c_void_p, C.c_void_p, _dp]
        L.qp_subproblem.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_double,
                                    _i64, _lp, _dp]
        L.qp_kkt.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, _dp]
        L.qp_norms.argtypes = [C.c_void_p, _dp, _dp]
        L.qp_spmv_schedule.argtypes = [_i64, _lp, _ip, _i64]
        L.qp_spmv_schedule.restype = _i64
        L.qp_batch_create.argtypes = [_i64, _lp, _lp, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp,
                                      C.c_char_p, _dp, _dp, C.POINTER(C.c_void_p)]
        L.qp_batch_solve.argtypes = [C.c_void_p, C.POINTER(QPParams)]
        L.qp_batch_result.argtypes = [C.c_void_p, _i64, _dp, _dp, C.POINTER(QPInfo)]
        L.qp_batch_statuses.argtypes = [C.c_void_p, _ip, _dp]
        L.qp_batch_times.argtypes = [C.c_void_p, _dp, _dp]
        L.qp_batch_destroy.argtypes = [C.c_void_p]
        L.qp_batch_destroy.restype = None
        L.qp_batch_solve_static.argtypes = [_i64, _lp, _lp, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp,
                                            C.c_char_p, _dp, _dp, C.POINTER(QPParams), C.c_void_p,
                                            _dp, _dp, _ip, C.POINTER(QPInfo)]
        L.qp_measure_gather_rate.argtypes = [_i64, _i64, C.c_int32, _dp]
        L.qp_batch_num_shapes.argtypes = []
        L.qp_batch_default_shape.argtypes = [C.c_int32]
        L.qp_batch_shape_info.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]
        L.qp_batch_set_schedule.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.qp_batch_get_schedule.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.qp_batch_tune.argtypes = [C.c_void_p, C.POINTER(QPParams), _dp]
        L.qp_server_config_default.restype = ServerConfig
        L.qp_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(QPParams), C.POINTER(C.c_void_p)]
        L.qp_server_submit.argtypes = [C.c_void_p, _i64, _i64, _lp, _ip, _dp, _lp, _ip, _dp, _dp, _dp,
                                       C.c_char_p, _dp, _dp]
        L.qp_server_submit.restype = _i64
        L.qp_server_wait.argtypes = [C.c_void_p, _i64, C.c_double]
        L.qp_server_result.argtypes = [C.c_void_p, _i64, _dp, _dp, C.POINTER(QPInfo),
                                       C.POINTER(RequestTimes)]
        L.qp_server_destroy.argtypes = [C.c_void_p]
        L.qp_server_destroy.restype = None
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


def _check(rc):
    if rc < 0:
        raise QPError(rc, qp_last_error())
    return rc


def _ptr(t):
    """Device pointer of a torch tensor (must be float64 and contiguous)."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return C.c_void_p(t.data_ptr())


# ---- the C ABI -------------------------------------------------------------------

def qp_params_default(**overrides) -> QPParams:
    p = lib().qp_params_default()
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def qp_last_error() -> str:
    return lib().qp_last_error().decode()


def qp_create(n, m, Q, A, c, b, sense: bytes, lb=None, ub=None):
    """Q, A: scipy CSR (Q may be None); returns an opaque handle."""
    qp_, qj_, qv_, keepq = _csr(Q)
    ap_, aj_, av_, keepa = _csr(A) if A is not None else (None, None, None, ())
    c, b, lb, ub = _f64(c), _f64(b), _f64(lb), _f64(ub)
    h = C.c_void_p()
    _check(lib().qp_create(n, m, qp_, qj_, qv_, ap_, aj_, av_, _d(c), _d(b), sense, _d(lb),
                           _d(ub), C.byref(h)))
    return h


def qp_create_ranged(n, m, Q, A, c, lc, uc, lb=None, ub=None):
    qp_, qj_, qv_, keepq = _csr(Q)
    ap_, aj_, av_, keepa = _csr(A) if A is not None else (None, None, None, ())
    c, lc, uc, lb, ub = _f64(c), _f64(lc), _f64(uc), _f64(lb), _f64(ub)
    h = C.c_void_p()
    _check(lib().qp_create_ranged(n, m, qp_, qj_, qv_, ap_, aj_, av_, _d(c), _d(lc), _d(uc),
                                  _d(lb), _d(ub), C.byref(h)))
    return h


def qp_create_factored(n, m, P, R, A, c, b, sense: bytes, lb=None, ub=None):
    """Q = P + R'R from its factors (P may be None; R k x n)."""
    pp_, pj_, pv_, keepp = _csr(P)
    rp_, rj_, rv_, keepr = _csr(R)
    ap_, aj_, av_, keepa = _csr(A) if A is not None else (None, None, None, ())
    c, b, lb, ub = _f64(c), _f64(b), _f64(lb), _f64(ub)
    h = C.c_void_p()
    _check(lib().qp_create_factored(n, m, pp_, pj_, pv_, R.shape[0], rp_, rj_, rv_, ap_, aj_, av_,
                                    _d(c), _d(b), sense, _d(lb), _d(ub), C.byref(h)))
    return h


def qp_create_from(qp):
    """Handle for a paper_2602_23967_amd.instances.QP (factored when qp.R is set)."""
    if getattr(qp, "R", None) is not None:
        return qp_create_factored(qp.n, qp.m, qp.Q, qp.R, qp.A, qp.c, qp.b, qp.sense, qp.lb, qp.ub)
    return qp_create(qp.n, qp.m, qp.Q, qp.A, qp.c, qp.b, qp.sense, qp.lb, qp.ub)


def qp_set_stream(h, stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t as int, or None."""
    raw = None if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    return _check(lib().qp_set_stream(h, C.c_void_p(raw)))


def qp_solve(h, tol=1e-6, max_iter=100000) -> int:
    return _check(lib().qp_solve(h, tol, max_iter))


def qp_solve_ex(h, params: QPParams | None = None) -> int:
    return _check(lib().qp_solve_ex(h, None if params is None else C.byref(params)))


def qp_result(h, n, m):
    """(status, x, y, info dict) of the last solve."""
    x = np.zeros(n)
    y = np.zeros(max(m, 1))
    info = QPInfo()
    st = _check(lib().qp_result(h, _d(x), _d(y), C.byref(info)))
    return st, x, y[:m], info.as_dict()


def qp_destroy(h):
    if h is not None and h.value:
        lib().qp_destroy(h)
        h.value = None


def qp_apply(h, op: int, x, y):
    return _check(lib().qp_apply(h, op, _ptr(x), _ptr(y)))


def qp_dot(h, a, b) -> float:
    out = C.c_double(0.0)
    _check(lib().qp_dot(h, a.numel(), _ptr(a), _ptr(b), C.byref(out)))
    return out.value


def qp_subproblem(h, tau, rhs, x, eps, max_inner=500):
    it = C.c_int64(0)
    res = C.c_double(0.0)
    _check(lib().qp_subproblem(h, tau, _ptr(rhs), _ptr(x), eps, max_inner, C.byref(it),
                               C.byref(res)))
    return it.value, res.value


def qp_kkt(h, x, y):
    out = (C.c_double * 7)()
    _check(lib().qp_kkt(h, _ptr(x), None if y is None else _ptr(y), out))
    return dict(zip(["r_primal", "r_dual", "r_gap", "pobj", "dobj", "natural", "pviol"], list(out)))


def qp_norms(h):
    a = C.c_double(0.0)
    q = C.c_double(0.0)
    _check(lib().qp_norms(h, C.byref(a), C.byref(q)))
    return a.value, q.value


def qp_spmv_schedule(rowptr):
    """(items, 8) int32 array of the SpMV schedule for a row-pointer array."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    rows = rp.shape[0] - 1
    k = _check(lib().qp_spmv_schedule(rows, rp.ctypes.data_as(_lp), None, 0))
    out = np.zeros((k, 8), dtype=np.int32)
    _check(lib().qp_spmv_schedule(rows, rp.ctypes.data_as(_lp), out.ctypes.data_as(_ip), k))
    return out


# ---- convenience -----------------------------------------------------------------

@dataclass
class Result:
    status: int
    x: np.ndarray
    y: np.ndarray
    info: dict

    @property
    def status_name(self):
        return STATUS_NAMES[self.status]


class Solver:
    """Owns one handle: Solver(qp).solve(tol=..., max_iter=...) -> Result."""

    def __init__(self, qp):
        self.qp = qp
        self.h = qp_create_from(qp)

    def solve(self, params: QPParams | None = None, **kw) -> Result:
        p = params if params is not None else qp_params_default(**kw)
        qp_solve_ex(self.h, p)
        st, x, y, info = qp_result(self.h, self.qp.n, self.qp.m)
        return Result(st, x, y, info)

    def close(self):
        qp_destroy(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched solve ----------------------------------------------------------------

def qp_batch_create(count, var_off, row_off, Q, A, c, b, sense: bytes, lb=None, ub=None):
    """Handle for `count` block-diagonally packed instances (see pdhcg.h)."""
    vo = np.ascontiguousarray(var_off, dtype=np.int64)
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    qp_, qj_, qv_, keepq = _csr(Q)
    ap_, aj_, av_, keepa = _csr(A) if A is not None else (None, None, None, ())
    c, b, lb, ub = _f64(c), _f64(b), _f64(lb), _f64(ub)
    h = C.c_void_p()
    _check(lib().qp_batch_create(count, vo.ctypes.data_as(_lp), ro.ctypes.data_as(_lp), qp_, qj_,
                                 qv_, ap_, aj_, av_, _d(c), _d(b), sense, _d(lb), _d(ub),
                                 C.byref(h)))
    return h


def qp_batch_solve(h, params: QPParams | None = None) -> int:
    return _check(lib().qp_batch_solve(h, None if params is None else C.byref(params)))


def qp_batch_result(h, i, n_i, m_i):
    x = np.zeros(n_i)
    y = np.zeros(max(m_i, 1))
    info = QPInfo()
    st = _check(lib().qp_batch_result(h, i, _d(x), _d(y), C.byref(info)))
    return st, x, y[:m_i], info.as_dict()


def qp_batch_statuses(h, count):
    st = np.zeros(count, dtype=np.int32)
    sec = C.c_double(0.0)
    _check(lib().qp_batch_statuses(h, st.ctypes.data_as(_ip), C.byref(sec)))
    return st, sec.value


def qp_batch_destroy(h):
    if h is not None and h.value:
        lib().qp_batch_destroy(h)
        h.value = None


STATIC_WORKSPACE_BYTES = 64 << 20   # QP_STATIC_WORKSPACE_BYTES


def qp_batch_solve_static(count, var_off, row_off, Q, A, c, b, sense: bytes, lb=None, ub=None,
                          params: QPParams | None = None, stream=None):
    """One blocking batched solve whose device memory is the library's
    static workspace (qp_batch_solve_static).  Returns (number of OPTIMAL
    instances, x, y, status per instance, info dict per instance)."""
    vo = np.ascontiguousarray(var_off, dtype=np.int64)
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    qp_, qj_, qv_, keepq = _csr(Q)
    ap_, aj_, av_, keepa = _csr(A) if A is not None else (None, None, None, ())
    c, b, lb, ub = _f64(c), _f64(b), _f64(lb), _f64(ub)
    n, m = int(vo[count]), int(ro[count])
    x = np.zeros(n)
    y = np.zeros(max(m, 1))
    st = np.zeros(count, dtype=np.int32)
    infos = (QPInfo * count)()
    s_ = None if stream is None else C.c_void_p(stream)
    opt = _check(lib().qp_batch_solve_static(count, vo.ctypes.data_as(_lp), ro.ctypes.data_as(_lp), qp_, qj_,
                                             qv_, ap_, aj_, av_, _d(c), _d(b), sense, _d(lb), _d(ub),
                                             None if params is None else C.byref(params), s_, _d(x), _d(y),
                                             st.ctypes.data_as(_ip), infos))
    return opt, x, y[:m], st, [infos[i].as_dict() for i in range(count)]


def qp_batch_num_shapes() -> int:
    return _check(lib().qp_batch_num_shapes())


def measure_gather_rate(n: int, gathers: int, repeats: int = 20) -> float:
    """Random 8-byte gathers per second from n doubles, XCD-keyed parts
    (qp_measure_gather_rate: a measurement utility, not part of the method)."""
    out = C.c_double(0.0)
    _check(lib().qp_measure_gather_rate(n, gathers, repeats, C.byref(out)))
    return out.value


def qp_batch_default_shape(general: bool = False) -> int:
    """Default launch shape of a batch (general: the one for non-diagonal-Q instances)."""
    return _check(lib().qp_batch_default_shape(1 if general else 0))


def qp_batch_shape_info(shape):
    """(threads per workgroup, LDS doubles, waves per SIMD) of a compiled batch shape."""
    t, l_, w = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    _check(lib().qp_batch_shape_info(shape, C.byref(t), C.byref(l_), C.byref(w)))
    return t.value, l_.value, w.value


def qp_batch_set_schedule(h, shape=-1, order=-1):
    _check(lib().qp_batch_set_schedule(h, shape, order))


def qp_batch_get_schedule(h):
    s_, o = C.c_int32(0), C.c_int32(0)
    _check(lib().qp_batch_get_schedule(h, C.byref(s_), C.byref(o)))
    return s_.value, o.value


def qp_batch_tune(h, params: QPParams | None = None):
    """Time every (shape, order) on the batch; returns (best candidate, seconds per candidate)."""
    sec = np.zeros(2 * qp_batch_num_shapes())
    best = _check(lib().qp_batch_tune(h, None if params is None else C.byref(params), _d(sec)))
    return best, sec


def batch_signature(qps, params: QPParams | None = None) -> str:
    """Key under which a tuned batch schedule is cached: instance count and
    largest n + m (both rounded up to powers of two), whether any instance
    has a non-diagonal Q, and the precision."""
    def up2(v):
        return 1 << max(0, int(v) - 1).bit_length()
    gen = any(q.Q is not None and not _is_diagonal(q.Q) for q in qps)
    prec = params.precision if params is not None else PRECISION_FP64
    return (f"count={up2(len(qps))};maxdim={up2(max(q.n + q.m for q in qps))};"
            f"general={int(gen)};precision={prec}")


def _is_diagonal(Q) -> bool:
    import scipy.sparse as sp
    Q = sp.csr_matrix(Q)
    r, c_ = Q.nonzero()
    return bool(np.all(r == c_))


def qp_batch_times(h, count):
    """(start, end) seconds of each instance of the last solve, after the
    first instance was taken up (device wall clock)."""
    t0 = np.zeros(count)
    t1 = np.zeros(count)
    _check(lib().qp_batch_times(h, _d(t0), _d(t1)))
    return t0, t1


class BatchSolver:
    """Owns a batch of instances.QP objects (diagonal or zero Q each)."""

    def __init__(self, qps):
        from .instances import pack
        self.qps = list(qps)
        big, self.var_off, self.row_off = pack(self.qps)
        self.h = qp_batch_create(len(self.qps), self.var_off, self.row_off, big.Q, big.A, big.c,
                                 big.b, big.sense, big.lb, big.ub)

    def solve(self, params: QPParams | None = None, **kw):
        p = params if params is not None else qp_params_default(**kw)
        qp_batch_solve(self.h, p)
        return qp_batch_statuses(self.h, len(self.qps))

    def result(self, i) -> Result:
        q = self.qps[i]
        st, x, y, info = qp_batch_result(self.h, i, q.n, q.m)
        return Result(st, x, y, info)

    def times(self):
        """(start, end) seconds of each instance of the last solve."""
        return qp_batch_times(self.h, len(self.qps))

    def set_schedule(self, shape=-1, order=-1):
        qp_batch_set_schedule(self.h, shape, order)

    def schedule(self):
        """(shape, order) of the next solve."""
        return qp_batch_get_schedule(self.h)

    def tune(self, params: QPParams | None = None, cache: str | None = None):
        """Pick the fastest launch schedule for this batch (qp_batch_tune).
        With `cache` (a JSON file), a schedule stored under this batch's
        signature is reused without timing, and a new one is stored.
        Returns {"shape", "order", "threads", "lds", "waves_per_simd",
        "seconds", "cached"}."""
        import json
        key = batch_signature(self.qps, params)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            e = table[key]
            self.set_schedule(e["shape"], e["order"])
            return dict(e, cached=True)
        best, sec = qp_batch_tune(self.h, params)
        shape, order = best // 2, best % 2
        threads, lds, waves = qp_batch_shape_info(shape)
        e = {"shape": shape, "order": order, "threads": threads, "lds": lds, "waves_per_simd": waves,
             "seconds": [float(v) for v in sec]}
        if cache:
            table[key] = e
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(e, cached=False)

    def close(self):
        qp_batch_destroy(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- request server ---------------------------------------------------------------

def qp_server_config_default(**overrides) -> ServerConfig:
    c = lib().qp_server_config_default()
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def qp_server_create(cfg: ServerConfig | None = None, params: QPParams | None = None):
    h = C.c_void_p()
    _check(lib().qp_server_create(None if cfg is None else C.byref(cfg),
                                  None if params is None else C.byref(params), C.byref(h)))
    return h


def qp_server_submit(h, n, m, Q, A, c, b, sense: bytes, lb=None, ub=None) -> int:
    qp_, qj_, qv_, keepq = _csr(Q)
    ap_, aj_, av_, keepa = _csr(A) if A is not None else (None, None, None, ())
    c, b, lb, ub = _f64(c), _f64(b), _f64(lb), _f64(ub)
    return _check(lib().qp_server_submit(h, n, m, qp_, qj_, qv_, ap_, aj_, av_, _d(c), _d(b), sense,
                                         _d(lb), _d(ub)))


def qp_server_wait(h, rid, timeout=-1.0) -> int:
    return _check(lib().qp_server_wait(h, rid, timeout))


def qp_server_result(h, rid, n, m):
    """(status, x, y, info dict, times dict) of a finished request (releases it)."""
    x = np.zeros(n)
    y = np.zeros(max(m, 1))
    info = QPInfo()
    times = RequestTimes()
    st = _check(lib().qp_server_result(h, rid, _d(x), _d(y), C.byref(info), C.byref(times)))
    return st, x, y[:m], info.as_dict(), times.as_dict()


def qp_server_destroy(h):
    if h is not None and h.value:
        lib().qp_server_destroy(h)
        h.value = None


class Server:
    """Request server: submit(qp) -> id, wait(id), result(id) -> (Result, times)."""

    def __init__(self, params: QPParams | None = None, **cfg):
        self.h = qp_server_create(qp_server_config_default(**cfg), params)
        self.shapes = {}

    def submit(self, qp) -> int:
        rid = qp_server_submit(self.h, qp.n, qp.m, qp.Q, qp.A, qp.c, qp.b, qp.sense, qp.lb, qp.ub)
        self.shapes[rid] = (qp.n, qp.m)
        return rid

    def wait(self, rid, timeout=-1.0) -> int:
        return qp_server_wait(self.h, rid, timeout)

    def result(self, rid):
        n, m = self.shapes.pop(rid)
        st, x, y, info, times = qp_server_result(self.h, rid, n, m)
        return Result(st, x, y, info), times

    def close(self):
        qp_server_destroy(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
