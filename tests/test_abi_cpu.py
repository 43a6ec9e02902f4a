"""C-ABI checks that need no GPU: the library loads and exports every
function include/pdhcg.h declares, parameters default to the paper's
constants, input validation rejects malformed problems before touching a
device, and the SpMV schedule covers every nonzero exactly once."""

import json
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2602_23967_amd as P
from paper_2602_23967_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdhcg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = P.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_params_default_paper_constants():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    p = P.qp_params_default()
    assert p.gamma_inner == g["gamma_inner"]["value"]
    assert p.eps_min == g["eps_min"]["value"]
    assert p.eta_scale == g["eta_scale"]["value"]
    assert p.tol == g["tol"]["value"]


def _bad(fn, code):
    with pytest.raises(P.QPError) as e:
        fn()
    assert e.value.code == code
    assert P.qp_last_error() != ""


def test_validation_errors():
    q = I.tiny(0, n=5, m=3)
    mk = lambda **kw: (lambda: P.qp_create(kw.get("n", q.n), kw.get("m", q.m), kw.get("Q", q.Q),
                                           kw.get("A", q.A), kw.get("c", q.c), kw.get("b", q.b),
                                           kw.get("sense", q.sense), kw.get("lb", q.lb),
                                           kw.get("ub", q.ub)))
    _bad(mk(n=0), P.ERR_INVALID_ARG)
    _bad(mk(lb=q.ub, ub=q.lb - 1.0), P.ERR_INVALID_ARG)                 # lb > ub
    _bad(mk(lb=np.full(q.n, np.inf)), P.ERR_INVALID_ARG)                # lb = +inf
    c = q.c.copy(); c[2] = np.nan
    _bad(mk(c=c), P.ERR_INVALID_ARG)
    b = q.b.copy(); b[0] = np.inf
    _bad(mk(b=b), P.ERR_INVALID_ARG)
    _bad(mk(sense=b"EXG"), P.ERR_INVALID_ARG)
    Qn = q.Q.toarray(); Qn[0, 1] += 1.0
    _bad(mk(Q=sp.csr_matrix(Qn)), P.ERR_NOT_SYMMETRIC)
    Qp = q.Q.toarray(); Qp[0, 4] = 0.0; Qp[4, 0] = 0.0
    Qs = sp.csr_matrix(Qp); Qs.eliminate_zeros()
    Qs = Qs.tolil(); Qs[0, 4] = 1.0; Qs = Qs.tocsr()
    _bad(mk(Q=Qs), P.ERR_NOT_SYMMETRIC)


def test_validation_raw_csr_errors():
    """Raw CSR arrays that scipy would normalise: unsorted / duplicate /
    out-of-range columns, decreasing row pointers, non-finite values."""
    import ctypes as C
    L = P.lib()
    n, m = 3, 2
    c = np.zeros(n)
    b = np.zeros(m)
    def call(ap, aj, av):
        ap = np.asarray(ap, np.int64); aj = np.asarray(aj, np.int32); av = np.asarray(av, np.float64)
        h = C.c_void_p()
        return L.qp_create(n, m, None, None, None, ap.ctypes.data_as(P._lp), aj.ctypes.data_as(P._ip),
                           av.ctypes.data_as(P._dp), c.ctypes.data_as(P._dp), b.ctypes.data_as(P._dp),
                           b"EE", None, None, C.byref(h))
    assert call([0, 2, 3], [1, 0, 2], [1, 1, 1]) == P.ERR_INVALID_ARG      # unsorted
    assert call([0, 2, 3], [1, 1, 2], [1, 1, 1]) == P.ERR_INVALID_ARG      # duplicate
    assert call([0, 2, 3], [0, 3, 2], [1, 1, 1]) == P.ERR_INVALID_ARG      # out of range
    assert call([0, 2, 1], [0, 1, 2], [1, 1, 1]) == P.ERR_INVALID_ARG      # decreasing
    assert call([1, 2, 3], [0, 1, 2], [1, 1, 1]) == P.ERR_INVALID_ARG      # rowptr[0] != 0
    assert call([0, 2, 3], [0, 1, 2], [1, np.nan, 1]) == P.ERR_INVALID_ARG
    assert call([0, 2, 3], [0, 1, 2], [1, np.inf, 1]) == P.ERR_INVALID_ARG


def test_ranged_validation():
    q = I.tiny(1, n=4, m=2)
    _bad(lambda: P.qp_create_ranged(q.n, q.m, q.Q, q.A, q.c, np.array([1.0, 0.0]),
                                    np.array([0.0, 1.0]), q.lb, q.ub), P.ERR_INVALID_ARG)
    _bad(lambda: P.qp_create_ranged(q.n, q.m, q.Q, q.A, q.c, np.array([np.inf, 0.0]),
                                    np.array([np.inf, 1.0]), q.lb, q.ub), P.ERR_INVALID_ARG)


def test_null_handle_calls():
    import ctypes as C
    L = P.lib()
    assert L.qp_solve(None, 1e-6, 10) == P.ERR_INVALID_ARG
    assert L.qp_result(None, None, None, None) == P.ERR_INVALID_ARG
    assert L.qp_set_stream(None, None) == P.ERR_INVALID_ARG
    L.qp_destroy(None)


@pytest.mark.parametrize("lengths", [
    [11] * 1000,                                   # short uniform rows
    [0, 0, 3, 0, 5000, 1, 2048, 2049, 0, 7] * 3,   # empty, one-block long and boundary rows
    [1] * 300 + [300] * 20 + [4097] + [0] * 5,     # row cap, medium rows, a one-block long row
    [3, 8192, 8193, 0, 20000, 2] * 2,              # the longest one-block row, segmented rows
    [],                                            # no rows
    [0] * 10,                                      # only empty rows
])
def test_spmv_schedule_covers_each_nonzero_once(lengths):
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    items = P.qp_spmv_schedule(rp)
    rows = len(lengths)
    seen_rows = np.zeros(rows, int)
    seen_nnz = np.zeros(int(rp[-1]), int)
    seg_slots = set()
    for row0, nr, k0, k1, lr, seg, nseg, base in items:
        assert 0 <= k1 - k0 <= 2048 or (nr == 1 and 2048 < k1 - k0 <= 8192)
        if nr > 0:
            assert nr <= 256
            assert k0 == rp[row0] and k1 == rp[row0 + nr]
            seen_rows[row0:row0 + nr] += 1
            seen_nnz[k0:k1] += 1
        elif nseg > 0:
            assert lengths[row0] > 8192 and 0 <= seg < nseg and k1 - k0 <= 2048
            assert rp[row0] <= k0 < k1 <= rp[row0 + 1]
            seen_nnz[k0:k1] += 1
            seg_slots.add(base + seg)
            if seg == 0:
                seen_rows[row0] += 1
        else:
            assert k0 == k1
    assert np.all(seen_rows == 1)
    assert np.all(seen_nnz == 1)
    assert seg_slots == set(range(len(seg_slots)))


def test_no_device_gives_device_error_or_success():
    """On a machine without a GPU, a valid problem passes validation and
    fails only at the device step; with a GPU it is created."""
    q = I.tiny(2, n=4, m=2)
    try:
        h = P.qp_create_from(q)
    except P.QPError as e:
        assert e.code == P.ERR_DEVICE
    else:
        P.qp_destroy(h)


def test_static_batch_without_a_device():
    """The allocation-free batched solve needs a device: without one it
    reports QP_ERR_DEVICE (with one, it solves)."""
    qs = [I.tiny_lp(1), I.tiny_lp(2)]
    big, vo, ro = I.pack(qs)
    try:
        opt, x, y, st, infos = P.qp_batch_solve_static(len(qs), vo, ro, big.Q, big.A, big.c, big.b, big.sense,
                                                       big.lb, big.ub)
    except P.QPError as e:
        assert e.code == P.ERR_DEVICE
    else:
        assert len(st) == 2 and x.shape == (big.n,)


def test_batch_validation_errors():
    from paper_2602_23967_amd.instances import pack
    qs = [I.mpc(i, horizon=10) for i in range(3)]
    big, vo, ro = pack(qs)
    mk = lambda **kw: (lambda: P.qp_batch_create(kw.get("count", 3), kw.get("vo", vo), kw.get("ro", ro),
                                                 kw.get("Q", big.Q), kw.get("A", big.A), big.c, big.b,
                                                 big.sense, big.lb, big.ub))
    _bad(mk(count=0), P.ERR_INVALID_ARG)
    vo2 = vo.copy(); vo2[1] = vo2[0]
    _bad(mk(vo=vo2), P.ERR_INVALID_ARG)                       # empty instance
    A2 = big.A.tolil(); A2[0, int(vo[1]) + 1] = 1.0           # entry outside its block
    _bad(mk(A=A2.tocsr()), P.ERR_INVALID_ARG)
    Qn = big.Q.tolil(); Qn[0, int(vo[1])] = 0.5; Qn[int(vo[1]), 0] = 0.5   # Q entry across blocks
    _bad(mk(Q=Qn.tocsr()), P.ERR_INVALID_ARG)
    Qs = big.Q.tolil(); Qs[0, 1] = 0.5                          # Q not symmetric
    _bad(mk(Q=Qs.tocsr()), P.ERR_NOT_SYMMETRIC)
    try:
        h = mk()()
    except P.QPError as e:
        assert e.code == P.ERR_DEVICE                          # no GPU here
    else:
        P.qp_batch_destroy(h)


def test_server_config_and_validation():
    c = P.qp_server_config_default()
    assert c.batch_lanes >= 1 and c.single_workers >= 1 and c.max_batch >= 1 and c.device_budget > 0
    import ctypes as C
    L = P.lib()
    h = C.c_void_p()
    bad = P.qp_server_config_default(batch_lanes=0, general_lanes=0, single_workers=0)
    assert L.qp_server_create(C.byref(bad), None, C.byref(h)) == P.ERR_INVALID_ARG
    bad = P.qp_server_config_default(max_batch=0)
    assert L.qp_server_create(C.byref(bad), None, C.byref(h)) == P.ERR_INVALID_ARG
    badp = P.qp_params_default(precision=3)
    assert L.qp_server_create(None, C.byref(badp), C.byref(h)) == P.ERR_INVALID_ARG
    assert L.qp_server_submit(None, 1, 0, None, None, None, None, None, None, None, None, None,
                              None, None) == P.ERR_INVALID_ARG
    assert L.qp_server_wait(None, 0, 0.0) == P.ERR_INVALID_ARG
    L.qp_server_destroy(None)
    rc = L.qp_server_create(None, None, C.byref(h))
    if rc == 0:                                   # a GPU is present
        L.qp_server_destroy(h)
    else:
        assert rc == P.ERR_DEVICE


def test_factored_validation():
    q = I.random_factored(0, n=20, m=5, k=3)
    mk = lambda R, k=None: (lambda: P.qp_create_factored(q.n, q.m, q.Q, R, q.A, q.c, q.b, q.sense,
                                                         q.lb, q.ub))
    R = q.R.tolil()
    R[0, 25 - 6] = 1.0                       # still in range: valid
    import ctypes as C
    L = P.lib()
    h = C.c_void_p()
    rp = np.ascontiguousarray(q.R.indptr, np.int64)
    rj = np.ascontiguousarray(q.R.indices, np.int32)
    rv = np.ascontiguousarray(q.R.data, np.float64)
    rj_bad = rj.copy(); rj_bad[0] = q.n                      # column out of range
    assert L.qp_create_factored(q.n, 0, None, None, None, 3, rp.ctypes.data_as(P._lp),
                                rj_bad.ctypes.data_as(P._ip), rv.ctypes.data_as(P._dp), None, None,
                                None, np.ascontiguousarray(q.c).ctypes.data_as(P._dp), None, None,
                                None, None, C.byref(h)) == P.ERR_INVALID_ARG
    assert L.qp_create_factored(q.n, 0, None, None, None, 0, rp.ctypes.data_as(P._lp),
                                rj.ctypes.data_as(P._ip), rv.ctypes.data_as(P._dp), None, None,
                                None, np.ascontiguousarray(q.c).ctypes.data_as(P._dp), None, None,
                                None, None, C.byref(h)) == P.ERR_INVALID_ARG   # k = 0
    try:
        hh = P.qp_create_from(q)
    except P.QPError as e:
        assert e.code == P.ERR_DEVICE
    else:
        P.qp_destroy(hh)


def test_batch_rejects_long_rows():
    """A row (of A, A' or Q) longer than QP_BATCH_MAX_ROW is refused before
    any device call: the batched kernel sums a row with one thread."""
    from paper_2602_23967_amd.instances import pack
    qs = [I.mpc(0, horizon=10), I.portfolio(0, n_assets=300, k_factors=3)]
    big, vo, ro = pack(qs)
    _bad(lambda: P.qp_batch_create(2, vo, ro, big.Q, big.A, big.c, big.b, big.sense, big.lb, big.ub),
         P.ERR_INVALID_ARG)
    assert "QP_BATCH_MAX_ROW" in P.qp_last_error()


def test_gather_rate_validation():
    import ctypes as C
    L = P.lib()
    out = C.c_double(0.0)
    for n, g, r in ((2, 4096, 1), (1000, 100, 1), (1000, 4096, 0)):
        assert L.qp_measure_gather_rate(n, g, r, C.byref(out)) == P.ERR_INVALID_ARG
    assert L.qp_measure_gather_rate(1000, 4096, 1, None) == P.ERR_INVALID_ARG


def test_batch_shape_table_and_schedule_validation():
    import ctypes as C
    ns = P.qp_batch_num_shapes()
    assert ns >= 2
    shapes = [P.qp_batch_shape_info(i) for i in range(ns)]
    assert shapes[P.qp_batch_default_shape(False)] == (256, 4992, 4)   # the default shape
    for t, l_, w in shapes:
        # whole wavefronts; staged operands leave room in the 160 KiB of LDS;
        # 1..8 waves per SIMD
        assert t % 64 == 0 and 64 <= t <= 1024 and 0 < l_ * 8 <= 128 * 1024 and 1 <= w <= 8
    assert len(set(shapes)) == ns
    for bad in (-1, ns):
        with pytest.raises(P.QPError):
            P.qp_batch_shape_info(bad)
    L = P.lib()
    assert L.qp_batch_set_schedule(None, 0, 0) == P.ERR_INVALID_ARG
    assert L.qp_batch_tune(None, None, None) == P.ERR_INVALID_ARG
    h = C.c_void_p()
    for kw in ({"batch_shape": ns}, {"batch_shape": -2}, {"batch_order": 2}):
        bad = P.qp_server_config_default(**kw)
        assert L.qp_server_create(C.byref(bad), None, C.byref(h)) == P.ERR_INVALID_ARG
    for kw in ({"general_shape": ns}, {"general_shape": -2}, {"diag_workers": -2},
               {"diag_workers": 5, "single_workers": 4}):
        bad = P.qp_server_config_default(**kw)
        assert L.qp_server_create(C.byref(bad), None, C.byref(h)) == P.ERR_INVALID_ARG
    c = P.qp_server_config_default()
    assert c.batch_shape == -1 and c.batch_order == -1 and c.general_shape == -1 and c.diag_workers == -1
    assert P.qp_batch_default_shape(False) == 12
    g = P.qp_batch_default_shape(True)
    assert 0 <= g < ns and P.qp_batch_shape_info(g)[0] >= 512
