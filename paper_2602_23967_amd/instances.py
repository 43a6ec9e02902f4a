"""Seeded synthetic convex-QP instances.

This module only draws problem data.  It holds none of the solver's
arithmetic: no bound mapping, no projections, no norms.  Both the HIP path
and the CPU oracle are fed from here, so it must stay free of anything either
of them computes.

A QP is stated as in the paper's problem statement (Section 2, eq. QP):

    minimize   1/2 x^T Q x + c^T x
    subject to A x (sense) b   row-wise, sense in {'E', 'G', 'L'}
               lb <= x <= ub

Q is stored as full symmetric CSR (both triangles) or None (Q = 0).
Every generator is seeded by ``SeedSequence([260223967, family, instance])``
so an instance is reproducible from its family id and instance id alone.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

SEED_ROOT = 260223967

# family ids used in the seed sequence
FAM_RANDOM_SMALL = 0      # n=1000 random sparse QP (B^T B + 1e-2 I)
FAM_LARGE_SPARSE = 1      # n=1e6 diagonally dominant sparse QP
FAM_PORTFOLIO = 2         # factor-model portfolio, diagonal Q
FAM_SERVED = 4            # request streams for the server (kinds, sizes, arrivals)
FAM_FACTORED = 5          # QPs with Q = P + R'R given by its factors
FAM_TINY = 10             # tiny QPs for brute-force pins
FAM_LP = 11               # tiny LPs (Q = 0)
FAM_EQ = 12               # equality-only, unboxed QPs (dense KKT pins)
FAM_MIXED = 13            # medium QPs with free, one-sided and fixed variables


@dataclass
class QP:
    """One problem instance in CSR form (int64 row pointers, int32 columns)."""

    n: int
    m: int
    Q: sp.csr_matrix | None
    A: sp.csr_matrix
    c: np.ndarray
    b: np.ndarray
    sense: bytes
    lb: np.ndarray
    ub: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)
    # Q = P + R'R given by its factors (Q then holds P, or None for P = 0)
    R: sp.csr_matrix | None = None

    def explicit_Q(self) -> sp.csr_matrix | None:
        """Q written out (P + R'R formed; only for small instances)."""
        if self.R is None:
            return self.Q
        RR = _csr(self.R.T @ self.R)
        return RR if self.Q is None else _csr(self.Q + RR)

    def explicit(self) -> "QP":
        """The same problem with Q written out."""
        return QP(n=self.n, m=self.m, Q=self.explicit_Q(), A=self.A, c=self.c, b=self.b,
                  sense=self.sense, lb=self.lb, ub=self.ub, name=self.name + "_explicit",
                  meta=self.meta)

    def csr_arrays(self, M):
        """(rowptr int64, col int32, val float64) of a CSR matrix, C-contiguous."""
        M = M.tocsr()
        M.sum_duplicates()
        M.sort_indices()
        return (np.ascontiguousarray(M.indptr, dtype=np.int64),
                np.ascontiguousarray(M.indices, dtype=np.int32),
                np.ascontiguousarray(M.data, dtype=np.float64))

    @property
    def nnz_Q(self) -> int:
        return 0 if self.Q is None else int(self.Q.nnz)

    @property
    def nnz_A(self) -> int:
        return int(self.A.nnz)


def rng_for(family: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, family, instance]))


def _csr(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    return M


def _sparse_normal(rng, rows, cols, density, scale=1.0):
    return sp.random(rows, cols, density=density, format="csr", random_state=rng,
                     data_rvs=lambda k: rng.normal(0.0, scale, size=k))


# ---------------------------------------------------------------------------
# the workload families
# ---------------------------------------------------------------------------

def random_small(instance: int = 0, n: int = 1000, m: int | None = None,
                 infeasible: bool = False) -> QP:
    """Tiny random convex QP: Q = B^T B + 1e-2 I with B (n/2 x n) at 0.5 %
    density, A (n/2 x n) at 1 % density, N(0,1) entries; first half of the
    rows '=', second half '>='; box [-1, 1]; b = A x0 with x0 ~ U(-0.5, 0.5),
    minus U(0, 0.1) slack on the '>=' rows.

    For n other than 1000 the per-row nonzero counts of the n=1000 case are
    kept (B: 5 per row, A: 10 per row), so that B^T B stays sparse.

    ``infeasible`` copies row 0 onto row 1 and sets b1 = b0 + 1 (both '=')
    so that no x satisfies both rows.
    """
    rng = rng_for(FAM_RANDOM_SMALL, instance)
    m = n // 2 if m is None else m
    dB = 0.005 if n == 1000 else 5.0 / n
    dA = 0.01 if n == 1000 else 10.0 / n
    B = _sparse_normal(rng, n // 2, n, dB)
    Q = _csr(B.T @ B + 1e-2 * sp.identity(n, format="csr"))
    A = _sparse_normal(rng, m, n, dA).tolil()
    c = rng.normal(size=n)
    x0 = rng.uniform(-0.5, 0.5, size=n)
    ne = m // 2
    sense = np.array([ord("E")] * ne + [ord("G")] * (m - ne), dtype=np.uint8)
    if infeasible:
        A[1, :] = A[0, :]
    A = _csr(A)
    b = A @ x0
    b[ne:] -= rng.uniform(0.0, 0.1, size=m - ne)
    if infeasible:
        b[1] = b[0] + 1.0
    return QP(n=n, m=m, Q=Q, A=A, c=c, b=b, sense=sense.tobytes(),
              lb=np.full(n, -1.0), ub=np.full(n, 1.0),
              name=f"random_small_n{n}" + ("_infeasible" if infeasible else ""),
              meta={"x0": x0})


def large_sparse(instance: int = 0, n: int = 1_000_000, m: int | None = None,
                 offdiag_pairs_per_row: int = 5, a_nnz_per_row: int = 8,
                 infeasible: bool = False) -> QP:
    """Large sparse QP: n variables, m = n/2 rows (first half '=', second half
    '>=').  Q: n*offdiag_pairs_per_row random (i, j), i != j, N(0,1) values,
    symmetrised (about 2*offdiag_pairs_per_row off-diagonals per row), with
    the diagonal set to the row's absolute off-diagonal sum + 0.1 (strictly
    diagonally dominant, hence SPD).  A: a_nnz_per_row distinct uniform
    columns per row, N(0,1).  Box [0, 10]; c ~ N(0,1); b = A x0, x0 ~ U(0,5).

    ``infeasible`` overwrites an '=' row r2 with '=' row r1 and sets
    b[r2] = b[r1] + 1.
    """
    rng = rng_for(FAM_LARGE_SPARSE, instance)
    m = n // 2 if m is None else m
    npair = n * offdiag_pairs_per_row
    i = rng.integers(0, n, size=npair)
    j = rng.integers(0, n - 1, size=npair)
    j = j + (j >= i)                       # uniform over j != i
    v = rng.normal(size=npair)
    S = sp.coo_matrix((v, (i, j)), shape=(n, n))
    Qoff = _csr(S + S.T)
    diag = np.asarray(abs(Qoff).sum(axis=1)).ravel() + 0.1
    Q = _csr(Qoff + sp.diags(diag))

    k = a_nnz_per_row
    cols = rng.integers(0, n, size=(m, k))
    while True:
        srt = np.sort(cols, axis=1)
        bad = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            break
        cols[bad] = rng.integers(0, n, size=(bad.size, k))
    vals = rng.normal(size=(m, k))
    rows = np.repeat(np.arange(m), k)
    A = sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(m, n))
    c = rng.normal(size=n)
    x0 = rng.uniform(0.0, 5.0, size=n)
    ne = m // 2
    sense = np.array([ord("E")] * ne + [ord("G")] * (m - ne), dtype=np.uint8)
    meta = {}
    if infeasible:
        r1, r2 = rng.choice(ne, size=2, replace=False)
        A = A.tolil()
        A[r2, :] = A[r1, :]
        meta["rows"] = (int(r1), int(r2))
    A = _csr(A)
    b = A @ x0
    if infeasible:
        r1, r2 = meta["rows"]
        b[r2] = b[r1] + 1.0
    return QP(n=n, m=m, Q=Q, A=A, c=c, b=b, sense=sense.tobytes(),
              lb=np.zeros(n), ub=np.full(n, 10.0),
              name=f"large_sparse_n{n}" + ("_infeasible" if infeasible else ""),
              meta=meta)


def portfolio(instance: int = 0, n_assets: int = 200_000, k_factors: int = 1000,
              f_density: float = 0.01, infeasible: bool = False) -> QP:
    """Factor-model portfolio QP with diagonal Q.  Variables: weights w
    (n_assets) then factor exposures f (k_factors).  Q = diag(d) on w,
    d ~ U(0.01, 0.1), and I on f.  Rows: F w - f = 0 (F at f_density,
    N(0, 0.1)), then the budget row sum(w) = 1.  0 <= w <= 0.01, f free.
    c = -mu on w with mu ~ N(0.05, 0.02), 0 on f.

    ``infeasible`` asks the budget row for 0.01 n_assets + 1, more than the
    box allows (certificate: the budget row's multiplier)."""
    rng = rng_for(FAM_PORTFOLIO, instance)
    na, k = n_assets, k_factors
    n = na + k
    d = rng.uniform(0.01, 0.1, size=na)
    Q = _csr(sp.diags(np.concatenate([d, np.ones(k)])))
    F = _sparse_normal(rng, k, na, f_density, 0.1)
    A = _csr(sp.vstack([sp.hstack([F, -sp.identity(k)]),
                        sp.hstack([sp.csr_matrix(np.ones((1, na))), sp.csr_matrix((1, k))])]))
    mu = rng.normal(0.05, 0.02, size=na)
    c = np.concatenate([-mu, np.zeros(k)])
    b = np.concatenate([np.zeros(k), [0.01 * na + 1.0 if infeasible else 1.0]])
    lb = np.concatenate([np.zeros(na), np.full(k, -np.inf)])
    ub = np.concatenate([np.full(na, 0.01), np.full(k, np.inf)])
    return QP(n=n, m=k + 1, Q=Q, A=A, c=c, b=b, sense=b"E" * (k + 1), lb=lb, ub=ub,
              name=f"portfolio_n{na}_k{k}" + ("_infeasible" if infeasible else ""))


def portfolio_factored(instance: int = 0, n_assets: int = 200_000, k_factors: int = 1000,
                       f_density: float = 0.01) -> QP:
    """The factor-model portfolio of `portfolio` posed without factor
    variables: Q = diag(d) + F'F given by its factors (P = diag(d), R = F),
    the budget row sum(w) = 1 as the only row, 0 <= w <= 0.01, c = -mu.  Its
    optimal w and objective are those of `portfolio` with the same seed
    (f = F w eliminated)."""
    q = portfolio(instance, n_assets, k_factors, f_density)
    na, k = n_assets, k_factors
    P = _csr(q.Q[:na, :na])
    F = _csr(q.A[:k, :na])
    A = _csr(q.A[k:, :na])
    return QP(n=na, m=1, Q=P, A=A, c=q.c[:na].copy(), b=np.array([1.0]), sense=b"E",
              lb=q.lb[:na].copy(), ub=q.ub[:na].copy(), name=f"portfolio_factored_n{na}_k{k}", R=F)


def random_factored(instance: int = 0, n: int = 400, m: int = 150, k: int = 12,
                    boxed: bool = True) -> QP:
    """QP with Q = P + R'R: P sparse symmetric with a dominant positive
    diagonal (about 4 off-diagonals per row), R (k x n) at 20 % density
    N(0,1); A (m x n) at 3 % density, first half '=', second half '>=';
    box [-1, 1] (or free when not `boxed`); b = A x0 - slack, x0 ~ U(-0.5, 0.5)."""
    rng = rng_for(FAM_FACTORED, instance)
    S = _sparse_normal(rng, n, n, 2.0 / n)
    off = _csr(S + S.T)
    off.setdiag(0.0)
    off.eliminate_zeros()
    P = _csr(off + sp.diags(np.asarray(abs(off).sum(axis=1)).ravel() + 0.05))
    R = _sparse_normal(rng, k, n, 0.2)
    A = _sparse_normal(rng, m, n, 0.03)
    x0 = rng.uniform(-0.5, 0.5, size=n)
    b = A @ x0
    ne = m // 2
    b[ne:] -= rng.uniform(0.0, 0.1, size=m - ne)
    sense = (b"E" * ne) + (b"G" * (m - ne))
    lb = np.full(n, -1.0) if boxed else np.full(n, -np.inf)
    ub = np.full(n, 1.0) if boxed else np.full(n, np.inf)
    return QP(n=n, m=m, Q=P, A=_csr(A), c=rng.normal(size=n), b=b, sense=sense, lb=lb, ub=ub,
              name=f"random_factored{instance}", R=_csr(R))


def served_stream(count: int, instance: int = 0, rate: float = 2000.0):
    """A seeded stream of `count` requests for the server: Poisson arrivals at
    `rate` per second; 60 % batched-MPC instances, 30 % random QPs of the
    random_small family with n ~ U{1000..50000} (per-row nonzeros held),
    10 % portfolios with n_assets ~ U{10000..100000} and max(1, n/200)
    factors; 2 % of the requests are the infeasible variant of their family.
    Returns (arrival offsets in seconds, list of QP)."""
    rng = rng_for(FAM_SERVED, instance)
    gaps = rng.exponential(1.0 / rate, size=count)
    kind = rng.choice(3, size=count, p=[0.6, 0.3, 0.1])
    bad = rng.random(count) < 0.02
    sizes = rng.integers(1000, 50001, size=count)
    assets = rng.integers(10000, 100001, size=count)
    qs = []
    for i in range(count):
        if kind[i] == 0:
            qs.append(mpc(1_000_000 + instance * count + i, infeasible=bool(bad[i])))
        elif kind[i] == 1:
            qs.append(random_small(1_000_000 + instance * count + i, n=int(sizes[i]),
                                   infeasible=bool(bad[i])))
        else:
            na = int(assets[i])
            qs.append(portfolio(1_000_000 + instance * count + i, n_assets=na,
                                k_factors=max(1, na // 200), infeasible=bool(bad[i])))
    return np.cumsum(gaps), qs


# ---------------------------------------------------------------------------
# small instances for pins and edge cases
# ---------------------------------------------------------------------------

def tiny(instance: int, n: int = 6, m: int = 3, density: float = 0.6,
         q_rank: int | None = None, boxed: bool = True, senses: str = "EGL") -> QP:
    """Tiny QP with a strictly convex Q = B^T B + 0.1 I (or rank-deficient
    B^T B when q_rank is given), a random A, a box [-1, 1] when boxed, and
    rows feasible at an interior point x0 ~ U(-0.5, 0.5)."""
    rng = rng_for(FAM_TINY, instance)
    r = n if q_rank is None else q_rank
    B = rng.normal(size=(r, n))
    Q = B.T @ B + (0.1 * np.eye(n) if q_rank is None else 0.0)
    A = rng.normal(size=(m, n)) * (rng.uniform(size=(m, n)) < density)
    for i in range(m):                     # no empty rows
        if not A[i].any():
            A[i, rng.integers(n)] = rng.normal()
    x0 = rng.uniform(-0.5, 0.5, size=n)
    sense = np.array([ord(senses[i % len(senses)]) for i in range(m)], dtype=np.uint8)
    b = A @ x0
    slack = rng.uniform(0.05, 0.3, size=m)
    b = np.where(sense == ord("G"), b - slack, np.where(sense == ord("L"), b + slack, b))
    c = rng.normal(size=n) * 2.0
    lb = np.full(n, -1.0) if boxed else np.full(n, -np.inf)
    ub = np.full(n, 1.0) if boxed else np.full(n, np.inf)
    return QP(n=n, m=m, Q=_csr(Q), A=_csr(A), c=c, b=b, sense=sense.tobytes(),
              lb=lb, ub=ub, name=f"tiny{instance}", meta={"x0": x0})


def tiny_lp(instance: int, n: int = 8, m: int = 4) -> QP:
    """Tiny bounded LP (Q = None): box [0, 2], rows feasible at x0 ~ U(0.5, 1.5)."""
    rng = rng_for(FAM_LP, instance)
    A = rng.normal(size=(m, n))
    x0 = rng.uniform(0.5, 1.5, size=n)
    sense = np.array([ord("EGL"[i % 3]) for i in range(m)], dtype=np.uint8)
    b = A @ x0
    b = np.where(sense == ord("G"), b - 0.2, np.where(sense == ord("L"), b + 0.2, b))
    c = rng.normal(size=n)
    return QP(n=n, m=m, Q=None, A=_csr(A), c=c, b=b, sense=sense.tobytes(),
              lb=np.zeros(n), ub=np.full(n, 2.0), name=f"tiny_lp{instance}")


def equality_qp(instance: int, n: int = 40, m: int = 15) -> QP:
    """Unboxed, equality-only strictly convex QP (X = R^n, S = {b})."""
    rng = rng_for(FAM_EQ, instance)
    B = rng.normal(size=(n, n)) * (rng.uniform(size=(n, n)) < 0.2)
    Q = B.T @ B / n + 0.5 * np.eye(n)
    A = rng.normal(size=(m, n)) * (rng.uniform(size=(m, n)) < 0.3)
    for i in range(m):
        if not A[i].any():
            A[i, rng.integers(n)] = 1.0
    b = rng.normal(size=m)
    c = rng.normal(size=n)
    return QP(n=n, m=m, Q=_csr(Q), A=_csr(A), c=c, b=b, sense=b"E" * m,
              lb=np.full(n, -np.inf), ub=np.full(n, np.inf), name=f"eq{instance}")


def mixed_bounds(instance: int, n: int = 300, m: int = 120) -> QP:
    """Medium sparse QP whose variables mix every bound kind: boxed, lower
    only, upper only, free, and fixed (l = u); rows mix '=', '>=', '<='.
    Feasible at x0 by construction."""
    rng = rng_for(FAM_MIXED, instance)
    B = _sparse_normal(rng, n // 2, n, 4.0 / n)
    Q = _csr(B.T @ B + 0.05 * sp.identity(n))
    A = _sparse_normal(rng, m, n, 6.0 / n).tolil()
    for i in range(m):
        if A.rows[i] == []:
            A[i, int(rng.integers(n))] = 1.0
    A = _csr(A)
    kind = rng.integers(0, 5, size=n)
    x0 = rng.uniform(-1.0, 1.0, size=n)
    lb = np.where((kind == 0) | (kind == 1), x0 - rng.uniform(0.1, 1.0, n), -np.inf)
    ub = np.where((kind == 0) | (kind == 2), x0 + rng.uniform(0.1, 1.0, n), np.inf)
    lb = np.where(kind == 4, x0, lb)
    ub = np.where(kind == 4, x0, ub)
    sense = np.array([ord("EGL"[i % 3]) for i in range(m)], dtype=np.uint8)
    b = A @ x0
    b = np.where(sense == ord("G"), b - 0.1, np.where(sense == ord("L"), b + 0.1, b))
    c = rng.normal(size=n)
    return QP(n=n, m=m, Q=Q, A=A, c=c, b=b, sense=sense.tobytes(), lb=lb, ub=ub,
              name=f"mixed{instance}")


def unbounded_qp(instance: int = 0, n: int = 12, m: int = 5) -> QP:
    """Dual-infeasible (unbounded) QP: variable 0 is free below, has zero
    curvature (row/column 0 of Q is zero), zero column in A, and c_0 > 0,
    so d = -e_0 is a ray with c^T d < 0, Q d = 0, A d = 0."""
    rng = rng_for(FAM_TINY, 1000 + instance)
    B = rng.normal(size=(n, n))
    Q = B.T @ B / n + 0.2 * np.eye(n)
    Q[0, :] = 0.0
    Q[:, 0] = 0.0
    A = rng.normal(size=(m, n))
    A[:, 0] = 0.0
    x0 = rng.uniform(-0.5, 0.5, size=n)
    b = A @ x0
    c = rng.normal(size=n)
    c[0] = 1.0
    lb = np.full(n, -1.0)
    ub = np.full(n, 1.0)
    lb[0] = -np.inf
    ub[0] = 1.0
    return QP(n=n, m=m, Q=_csr(Q), A=_csr(A), c=c, b=b, sense=b"E" * m, lb=lb, ub=ub,
              name=f"unbounded{instance}")


def contradictory_rows(instance: int = 0, n: int = 10, m: int = 4) -> QP:
    """Primal-infeasible QP: rows 0 and 1 have the same coefficients and
    right-hand sides b and b + 1 (both '='), so y = e_0 - e_1 (or its
    negative) is a Farkas ray."""
    q = tiny(2000 + instance, n=n, m=m, senses="E")
    A = q.A.toarray()
    A[1] = A[0]
    b = q.b.copy()
    b[1] = b[0] + 1.0
    q.A = _csr(A)
    q.b = b
    q.name = f"contradictory{instance}"
    return q


def box_infeasible_rows(instance: int = 0, n: int = 8, m: int = 3) -> QP:
    """Primal-infeasible through the box: row 0 asks sum(x) >= n + 1 while
    every x_i <= 1."""
    q = tiny(3000 + instance, n=n, m=m, senses="E")
    A = q.A.toarray()
    A[0] = 1.0
    b = q.b.copy()
    b[0] = n + 1.0
    s = bytearray(q.sense)
    s[0] = ord("G")
    q.A = _csr(A)
    q.b = b
    q.sense = bytes(s)
    q.name = f"box_infeasible{instance}"
    return q


FAM_MPC = 3


def mpc(instance: int = 0, horizon: int | None = None, infeasible: bool = False) -> QP:
    """Linear MPC QP over a horizon T ~ U{10..50}: states x_0..x_T (12 each),
    inputs u_0..u_{T-1} (4 each).  Rows: x_0 = x_init (12 '='), then
    x_{t+1} - A_d x_t - B_d u_t = 0 (12 '=' rows per step, 17 nonzeros each).
    A_d = U diag(lam) U' with U a random orthogonal matrix and lam ~ U(-0.95,
    0.95) rescaled so max |lam| = 0.95; B_d ~ N(0, 0.3).  Q = I on states,
    0.1 I on inputs, c = 0.  Bounds |u| <= 1, |x| <= 5; x_init ~ U(-1, 1).
    Variables are ordered x_0, u_0, x_1, u_1, ..., x_T.
    ``infeasible`` sets x_init[0] = 6, outside the state box."""
    rng = rng_for(FAM_MPC, instance)
    T = int(rng.integers(10, 51)) if horizon is None else int(horizon)
    ns, nu = 12, 4
    G = rng.normal(size=(ns, ns))
    U, _ = np.linalg.qr(G)
    lam = rng.uniform(-0.95, 0.95, size=ns)
    lam *= 0.95 / np.abs(lam).max()
    Ad = U @ np.diag(lam) @ U.T
    Bd = rng.normal(0.0, 0.3, size=(ns, nu))
    xinit = rng.uniform(-1.0, 1.0, size=ns)
    if infeasible:
        xinit[0] = 6.0
    step = ns + nu
    n = step * T + ns
    xo = lambda t: t * step              # offset of x_t
    uo = lambda t: t * step + ns         # offset of u_t
    rows, cols, vals = [], [], []
    for i in range(ns):                  # x_0 = x_init
        rows.append(i); cols.append(xo(0) + i); vals.append(1.0)
    r = ns
    for t in range(T):
        for i in range(ns):
            rows += [r] * (1 + ns + nu)
            cols += [xo(t + 1) + i] + [xo(t) + j for j in range(ns)] + [uo(t) + k for k in range(nu)]
            vals += [1.0] + list(-Ad[i]) + list(-Bd[i])
            r += 1
    m = r
    A = _csr(sp.csr_matrix((vals, (rows, cols)), shape=(m, n)))
    qd = np.ones(n)
    for t in range(T):
        qd[uo(t):uo(t) + nu] = 0.1
    lb = np.full(n, -5.0)
    ub = np.full(n, 5.0)
    for t in range(T):
        lb[uo(t):uo(t) + nu] = -1.0
        ub[uo(t):uo(t) + nu] = 1.0
    b = np.zeros(m)
    b[:ns] = xinit
    return QP(n=n, m=m, Q=_csr(sp.diags(qd)), A=A, c=np.zeros(n), b=b, sense=b"E" * m,
              lb=lb, ub=ub, name=f"mpc{instance}_T{T}" + ("_infeasible" if infeasible else ""),
              meta={"T": T, "xinit": xinit})


def pack(qps):
    """Block-diagonal packing of several QPs (one problem whose variables and
    rows are the instances' in order).  Returns (QP, var_off, row_off)."""
    var_off = np.zeros(len(qps) + 1, dtype=np.int64)
    row_off = np.zeros(len(qps) + 1, dtype=np.int64)
    for i, q in enumerate(qps):
        var_off[i + 1] = var_off[i] + q.n
        row_off[i + 1] = row_off[i] + q.m
    Qs = [q.Q.tocoo() if q.Q is not None else sp.coo_matrix((q.n, q.n)) for q in qps]
    Q = _csr(sp.block_diag(Qs, format="coo"))
    A = _csr(sp.block_diag([q.A.tocoo() for q in qps], format="coo"))
    qp = QP(n=int(var_off[-1]), m=int(row_off[-1]), Q=Q, A=A,
            c=np.concatenate([q.c for q in qps]), b=np.concatenate([q.b for q in qps]),
            sense=b"".join(q.sense for q in qps),
            lb=np.concatenate([q.lb for q in qps]), ub=np.concatenate([q.ub for q in qps]),
            name=f"pack{len(qps)}")
    return qp, var_off, row_off
