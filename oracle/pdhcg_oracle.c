/*
 * pdhcg_oracle.c -- plain, slow, FP64 CPU reference of PDHCG-II.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg, never by the product library.  It shares
 * no code with the HIP path.  Every loop is written out plainly; reductions
 * sum fixed 4096-element chunks in chunk order, so results do not depend on
 * the number of OpenMP threads.  Build flags: -O2 -ffp-contract=off, no
 * fast-math.
 *
 * What each part follows, and what pins it (tests/test_oracle_*.py):
 *   problem data, sign sets Y and R, p(z;l,u) ..... Section 2, eq. QP/dualQP
 *       pinned by algebraic identities (Moreau, idempotence, support of a box)
 *   PDHG step ....................................... Section 2.1, eq. pdhcg_update
 *   primal subproblem ............................... Section 2.2
 *       closed form (diagonal Q); CG on the free set with expansion and
 *       proportioning steps (MPRGP, Dostal & Schoeberl 2005) for a
 *       non-diagonal Q, plain CG when no bound is finite; projected gradient
 *       with Barzilai-Borwein steps as an independent second solver.
 *       pinned by numpy.linalg.solve (unboxed) and 3^n enumeration (boxed)
 *   reflected Halpern averaging ..................... Section 3.1
 *       pinned by its limit without restarts: the projection of the anchor
 *       onto the solution set (Wittmann), found by enumeration on LPs whose
 *       solution set is a face
 *   tau = eta/omega, sigma = eta*omega, eta = 0.998/||A|| ... Section 3.2
 *       ||A||_2 pinned by a dense SVD
 *   PID primal weight update ........................ Section 3.2, eq. pid
 *   adaptive inner tolerance ........................ Section 3.3
 *       restart / PID / tolerance trajectory: parity unpinned (the paper
 *       prints no trace); only their algebra on hand values is pinned
 *   KKT residuals r_primal, r_dual, r_gap ........... Section 4
 *       pinned by exact solutions (all three vanish) and by hand-worked exact
 *       values with nonzero numerators, each term of the r_dual and r_gap
 *       denominators dominating in turn
 *   primal / dual infeasibility certificates ........ Section 5
 *       pinned by constructed infeasible / unbounded instances with known rays
 *   final solutions ............................... dense KKT solves,
 *       active-set enumeration, scipy HiGHS on LPs
 *
 * Readings where the paper is silent or garbled (restart rule, Halpern
 * form, PID gains, tolerances of the certificates, ...) are listed with the
 * parameter defaults in oracle_params_default().
 */
#include "pdhcg_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHUNK 4096

/* wall clock in seconds (phase timings of oracle_info only) */
static double wall_seconds(void)
{
    struct timespec ts;
    timespec_get(&ts, TIME_UTC);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* parameters                                                                */
/* ------------------------------------------------------------------------ */

void oracle_params_default(oracle_params* p)
{
    memset(p, 0, sizeof(*p));
    p->tol = 1e-6;
    p->max_iter = 100000;
    p->check_every = 64;          /* reading: cadence of KKT/restart checks */
    p->max_inner = 500;           /* reading: inner iteration cap */
    p->inner_solver = ORACLE_INNER_AUTO;
    p->use_halpern = 1;
    p->theta = 1.0;               /* reading: Halpern on (1+theta)T - theta I */
    p->kp = 0.99;                 /* reading: PID gains (Section 3.2 gives none) */
    p->ki = 0.01;
    p->kd = 0.0;
    p->gamma_inner = 5e-4;        /* Section 3.3 */
    p->eps_min = 1e-9;            /* Section 3.3 */
    p->eps_inner_fixed = 0.0;
    p->restart_sufficient = 0.2;  /* reading: restart rule (not in the paper) */
    p->restart_necessary = 0.8;
    p->restart_artificial = 0.36;
    p->eps_inf = 1e-8;            /* reading: certificate tolerance */
    p->eta_scale = 0.998;         /* Section 3.2 */
    p->norm_safety = 1.01;        /* reading: guard against power-iteration underestimate */
    p->power_tol = 1e-7;
    p->power_max_iter = 1000;
    p->mprgp_gamma = 1.0;
    p->mprgp_abar_scale = 1.9;
    p->verbose = 0;
}

int oracle_bounds_from_sense(int64_t m, const double* b, const char* sense,
                             double* lc, double* uc)
{
    for (int64_t i = 0; i < m; ++i) {
        switch (sense[i]) {
        case 'E': lc[i] = b[i]; uc[i] = b[i]; break;
        case 'G': lc[i] = b[i]; uc[i] = INFINITY; break;
        case 'L': lc[i] = -INFINITY; uc[i] = b[i]; break;
        default: return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 at counter i (seed 0): the state after i+1 increments by the   */
/* golden-ratio constant, passed through the published mixing function.     */
/* ------------------------------------------------------------------------ */

double oracle_splitmix_unit(uint64_t i)
{
    uint64_t z = (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* plain vector and CSR kernels                                              */
/* ------------------------------------------------------------------------ */

static int64_t nchunks(int64_t n) { return (n + CHUNK - 1) / CHUNK; }

static double chunk_total(const double* part, int64_t nc)
{
    double s = 0.0;
    for (int64_t ch = 0; ch < nc; ++ch) s += part[ch];
    return s;
}

static double dot(int64_t n, const double* a, const double* b)
{
    int64_t nc = nchunks(n);
    double* part = (double*)calloc((size_t)(nc + 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < nc; ++ch) {
        int64_t lo = ch * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
        part[ch] = s;
    }
    double s = chunk_total(part, nc);
    free(part);
    return s;
}

static double nrm2(int64_t n, const double* a) { return sqrt(dot(n, a, a)); }

static double amax(int64_t n, const double* a)
{
    double r = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = fabs(a[i]);
        if (v > r || v != v) r = v;
        if (r != r) return r;
    }
    return r;
}

/* max |a_i| over finite entries only (0 when there are none) */
static double amax_finite(int64_t n, const double* a)
{
    double r = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (isfinite(a[i]) && fabs(a[i]) > r) r = fabs(a[i]);
    return r;
}

void oracle_csr_matvec(int64_t r, const int64_t* rowptr, const int32_t* col,
                       const double* val, const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < r; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* u = M' w by a sequential scatter (order fixed) */
static void csr_tmatvec(int64_t r, int64_t c, const int64_t* rowptr, const int32_t* col,
                        const double* val, const double* w, double* u)
{
    for (int64_t j = 0; j < c; ++j) u[j] = 0.0;
    for (int64_t i = 0; i < r; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) u[col[k]] += val[k] * w[i];
}

/* ------------------------------------------------------------------------ */
/* problem                                                                   */
/* ------------------------------------------------------------------------ */

enum { QK_NONE = 0, QK_DIAG = 1, QK_GENERAL = 2 };

typedef struct {
    int64_t n, m;
    const int64_t* Qp; const int32_t* Qj; const double* Qv;
    int qkind;
    double* qdiag;                          /* n; used when qkind != QK_GENERAL */
    const int64_t* Ap; const int32_t* Aj; const double* Av;
    int64_t* Tp; int32_t* Tj; double* Tv;   /* A transposed, n x m CSR */
    const double *c, *lc, *uc, *lv, *uv;
} oprob;

static int q_kind(int64_t n, const int64_t* Qp, const int32_t* Qj)
{
    if (!Qp) return QK_NONE;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = Qp[i]; k < Qp[i + 1]; ++k)
            if (Qj[k] != i) return QK_GENERAL;
    return QK_DIAG;
}

static void build_transpose(oprob* pr)
{
    int64_t n = pr->n, m = pr->m, nnz = pr->Ap[m];
    pr->Tp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    pr->Tj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    pr->Tv = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t k = 0; k < nnz; ++k) pr->Tp[pr->Aj[k] + 1]++;
    for (int64_t j = 0; j < n; ++j) pr->Tp[j + 1] += pr->Tp[j];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(fill, pr->Tp, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = pr->Ap[i]; k < pr->Ap[i + 1]; ++k) {
            int64_t d = fill[pr->Aj[k]]++;
            pr->Tj[d] = (int32_t)i;
            pr->Tv[d] = pr->Av[k];
        }
    free(fill);
}

static void setup_problem(oprob* pr, int64_t n, int64_t m,
                          const int64_t* Qp, const int32_t* Qj, const double* Qv,
                          const int64_t* Ap, const int32_t* Aj, const double* Av,
                          const double* c, const double* lc, const double* uc,
                          const double* lv, const double* uv)
{
    memset(pr, 0, sizeof(*pr));
    pr->n = n; pr->m = m;
    pr->Qp = Qp; pr->Qj = Qj; pr->Qv = Qv;
    pr->Ap = Ap; pr->Aj = Aj; pr->Av = Av;
    pr->c = c; pr->lc = lc; pr->uc = uc; pr->lv = lv; pr->uv = uv;
    pr->qkind = q_kind(n, Qp, Qj);
    pr->qdiag = (double*)calloc((size_t)n, sizeof(double));
    if (pr->qkind == QK_DIAG)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = Qp[i]; k < Qp[i + 1]; ++k) pr->qdiag[i] += Qv[k];
    build_transpose(pr);
}

static void free_problem(oprob* pr)
{
    free(pr->qdiag); free(pr->Tp); free(pr->Tj); free(pr->Tv);
}

static void qmul(const oprob* pr, const double* x, double* y)
{
    int64_t n = pr->n;
    if (pr->qkind == QK_GENERAL) {
        oracle_csr_matvec(n, pr->Qp, pr->Qj, pr->Qv, x, y);
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) y[i] = pr->qdiag[i] * x[i];
    }
}

static void amul(const oprob* pr, const double* x, double* y)
{
    oracle_csr_matvec(pr->m, pr->Ap, pr->Aj, pr->Av, x, y);
}

static void atmul(const oprob* pr, const double* y, double* x)
{
    oracle_csr_matvec(pr->n, pr->Tp, pr->Tj, pr->Tv, y, x);
}

/* y = (Q + I/tau) x */
static void hmul(const oprob* pr, double inv_tau, const double* x, double* y)
{
    qmul(pr, x, y);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < pr->n; ++i) y[i] += inv_tau * x[i];
}

/* ------------------------------------------------------------------------ */
/* sets of Section 2: projections and the support function                   */
/* ------------------------------------------------------------------------ */

static double clampd(double v, double l, double u) { return v < l ? l : (v > u ? u : v); }

/* proj onto the box [l, u] */
static void proj_box(int64_t k, const double* v, const double* l, const double* u, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < k; ++i) out[i] = clampd(v[i], l[i], u[i]);
}

/* Y_i: {0} free row, R+ upper only, R- lower only, R both */
static double proj_Y1(double v, double lc, double uc)
{
    int lf = isfinite(lc), uf = isfinite(uc);
    if (!lf && !uf) return 0.0;
    if (!lf) return v > 0.0 ? v : 0.0;
    if (!uf) return v < 0.0 ? v : 0.0;
    return v;
}

/* R_i: {0} free variable, R- upper only, R+ lower only, R both */
static double proj_R1(double v, double lv, double uv)
{
    int lf = isfinite(lv), uf = isfinite(uv);
    if (!lf && !uf) return 0.0;
    if (!lf) return v < 0.0 ? v : 0.0;
    if (!uf) return v > 0.0 ? v : 0.0;
    return v;
}

/* recession cone of the box [l, u]: {0} both finite, R+ lower only,
 * R- upper only, R free */
static double proj_rec1(double v, double l, double u)
{
    int lf = isfinite(l), uf = isfinite(u);
    if (lf && uf) return 0.0;
    if (lf) return v > 0.0 ? v : 0.0;
    if (uf) return v < 0.0 ? v : 0.0;
    return v;
}

/* p(z; l, u) = u'z^+ - l'z^-; a zero part contributes nothing (0*inf = 0) */
double oracle_support(int64_t k, const double* z, const double* l, const double* u)
{
    int64_t nc = nchunks(k);
    double* part = (double*)calloc((size_t)(nc + 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < nc; ++ch) {
        int64_t lo = ch * CHUNK, hi = lo + CHUNK < k ? lo + CHUNK : k;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) {
            if (z[i] > 0.0) s += u[i] * z[i];
            else if (z[i] < 0.0) s -= l[i] * (-z[i]);
        }
        part[ch] = s;
    }
    double s = chunk_total(part, nc);
    free(part);
    return s;
}

/* ------------------------------------------------------------------------ */
/* power iteration for ||M||_2                                              */
/* ------------------------------------------------------------------------ */

double oracle_norm2(int64_t r, int64_t c, const int64_t* rowptr, const int32_t* col,
                    const double* val, double tol, int64_t max_iter, int64_t* iters)
{
    if (iters) *iters = 0;
    if (r <= 0 || c <= 0 || rowptr[r] == 0) return 0.0;
    double* v = (double*)malloc(sizeof(double) * (size_t)c);
    double* w = (double*)malloc(sizeof(double) * (size_t)r);
    double* u = (double*)malloc(sizeof(double) * (size_t)c);
    for (int64_t j = 0; j < c; ++j) v[j] = 2.0 * oracle_splitmix_unit((uint64_t)j) - 1.0;
    double nv = nrm2(c, v);
    for (int64_t j = 0; j < c; ++j) v[j] /= nv;
    double sig = 0.0, prev = 0.0;
    int64_t it = 0;
    for (it = 1; it <= max_iter; ++it) {
        oracle_csr_matvec(r, rowptr, col, val, v, w);
        sig = nrm2(r, w);
        if (sig == 0.0) break;
        csr_tmatvec(r, c, rowptr, col, val, w, u);
        double nu = nrm2(c, u);
        if (nu == 0.0) break;
        for (int64_t j = 0; j < c; ++j) v[j] = u[j] / nu;
        if (fabs(sig - prev) <= tol * sig) break;
        prev = sig;
    }
    if (iters) *iters = it;
    free(v); free(w); free(u);
    return sig;
}

/* ------------------------------------------------------------------------ */
/* primal subproblem solvers (Section 2.2)                                   */
/*   minimise 1/2 x'Hx - rhs'x over lv <= x <= uv, H = Q + I/tau            */
/* ------------------------------------------------------------------------ */

/* Split of the gradient g at a feasible x (Dostal's notation):
 *   free set F = {l < x < u};  phi = g on F, 0 elsewhere;
 *   beta = min(g,0) at a lower bound, max(g,0) at an upper bound, 0 for a
 *   fixed variable (l = u);  reduced free gradient phit caps phi at the
 *   distance to the bound the step abar would cross.
 * The projected gradient is phi + beta. */
static void grad_split(int64_t n, const double* x, const double* g,
                       const double* l, const double* u, double abar,
                       double* phi, double* beta, double* phit)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double f = 0.0, b = 0.0, ft = 0.0;
        if (x[i] > l[i] && x[i] < u[i]) {
            f = g[i];
            if (g[i] > 0.0) ft = isfinite(l[i]) ? fmin((x[i] - l[i]) / abar, g[i]) : g[i];
            else if (g[i] < 0.0) ft = isfinite(u[i]) ? fmax((x[i] - u[i]) / abar, g[i]) : g[i];
        } else if (l[i] < u[i]) {
            if (x[i] <= l[i]) b = g[i] < 0.0 ? g[i] : 0.0;
            else b = g[i] > 0.0 ? g[i] : 0.0;
        }
        phi[i] = f; beta[i] = b; if (phit) phit[i] = ft;
    }
}

/* largest a >= 0 with l <= x - a*p <= u */
static double feasible_step(int64_t n, const double* x, const double* p,
                            const double* l, const double* u)
{
    double a = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double s = INFINITY;
        if (p[i] > 0.0 && isfinite(l[i])) s = (x[i] - l[i]) / p[i];
        else if (p[i] < 0.0 && isfinite(u[i])) s = (x[i] - u[i]) / p[i];
        if (s < a) a = s;
    }
    return a < 0.0 ? 0.0 : a;
}

/* x <- x - a*p, g <- g - a*Hp, then x clipped to the box against rounding */
static void step_xg(int64_t n, double a, const double* p, const double* Hp,
                    double* x, double* g, const double* l, const double* u)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        x[i] = clampd(x[i] - a * p[i], l[i], u[i]);
        g[i] -= a * Hp[i];
    }
}

static void gradient(const oprob* pr, double inv_tau, const double* x, const double* rhs, double* g)
{
    hmul(pr, inv_tau, x, g);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < pr->n; ++i) g[i] -= rhs[i];
}

/* ||g^P||_2 at feasible x */
static double proj_grad_norm(const oprob* pr, double inv_tau, const double* x, const double* rhs)
{
    int64_t n = pr->n;
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    double* phi = (double*)malloc(sizeof(double) * (size_t)n);
    double* beta = (double*)malloc(sizeof(double) * (size_t)n);
    gradient(pr, inv_tau, x, rhs, g);
    grad_split(n, x, g, pr->lv, pr->uv, 1.0, phi, beta, NULL);
    double r = sqrt(dot(n, phi, phi) + dot(n, beta, beta));
    free(g); free(phi); free(beta);
    return r;
}

static void closed_form(const oprob* pr, double inv_tau, const double* rhs, double* x)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < pr->n; ++i)
        x[i] = clampd(rhs[i] / (pr->qdiag[i] + inv_tau), pr->lv[i], pr->uv[i]);
}

/* MPRGP: conjugate gradients on the free set, with an expansion step
 * (feasible half step, then a projected step of length abar along the free
 * gradient) when the CG step would leave the box, and a proportioning step
 * along the chopped gradient when it dominates (||beta||^2 > Gam^2 phit'phi).
 * With no finite bound it is plain CG (Hestenes-Stiefel form). */
static int64_t mprgp(const oprob* pr, double inv_tau, const double* rhs, double* x,
                     double eps, int64_t max_inner, double Gam, double abar, double* res_out)
{
    int64_t n = pr->n;
    const double *l = pr->lv, *u = pr->uv;
    size_t bytes = sizeof(double) * (size_t)n;
    double* g = (double*)malloc(bytes);
    double* p = (double*)malloc(bytes);
    double* Hp = (double*)malloc(bytes);
    double* phi = (double*)malloc(bytes);
    double* beta = (double*)malloc(bytes);
    double* phit = (double*)malloc(bytes);

    proj_box(n, x, l, u, x);
    gradient(pr, inv_tau, x, rhs, g);
    grad_split(n, x, g, l, u, abar, phi, beta, phit);
    double b2 = dot(n, beta, beta);
    double gp2 = dot(n, phi, phi) + b2;
    double ptp = dot(n, phit, phi);
    memcpy(p, phi, bytes);

    int64_t it = 0;
    while (sqrt(gp2) > eps && it < max_inner) {
        ++it;
        if (b2 <= Gam * Gam * ptp) {
            hmul(pr, inv_tau, p, Hp);
            double pHp = dot(n, p, Hp);
            if (!(pHp > 0.0)) break;
            double acg = dot(n, g, p) / pHp;
            double af = feasible_step(n, x, p, l, u);
            if (acg <= af) {
                /* conjugate gradient step */
                step_xg(n, acg, p, Hp, x, g, l, u);
                grad_split(n, x, g, l, u, abar, phi, beta, phit);
                double gam = dot(n, phi, Hp) / pHp;
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) p[i] = phi[i] - gam * p[i];
            } else {
                /* expansion step */
                step_xg(n, af, p, Hp, x, g, l, u);
                grad_split(n, x, g, l, u, abar, phi, beta, phit);
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) x[i] = clampd(x[i] - abar * phi[i], l[i], u[i]);
                gradient(pr, inv_tau, x, rhs, g);
                grad_split(n, x, g, l, u, abar, phi, beta, phit);
                memcpy(p, phi, bytes);
            }
        } else {
            /* proportioning step along the chopped gradient */
            memcpy(p, beta, bytes);
            hmul(pr, inv_tau, p, Hp);
            double dHd = dot(n, p, Hp);
            if (!(dHd > 0.0)) break;
            double a = dot(n, g, p) / dHd;
            double af = feasible_step(n, x, p, l, u);
            if (af < a) a = af;
            step_xg(n, a, p, Hp, x, g, l, u);
            grad_split(n, x, g, l, u, abar, phi, beta, phit);
            memcpy(p, phi, bytes);
        }
        b2 = dot(n, beta, beta);
        gp2 = dot(n, phi, phi) + b2;
        ptp = dot(n, phit, phi);
    }
    if (res_out) *res_out = sqrt(gp2);
    free(g); free(p); free(Hp); free(phi); free(beta); free(phit);
    return it;
}

/* Projected gradient with Barzilai-Borwein step lengths (first BB formula)
 * and a non-monotone Armijo safeguard over the last 10 objective values. */
static int64_t bbpg(const oprob* pr, double inv_tau, const double* rhs, double* x,
                    double eps, int64_t max_inner, double norm_Q, double* res_out)
{
    int64_t n = pr->n;
    const double *l = pr->lv, *u = pr->uv;
    size_t bytes = sizeof(double) * (size_t)n;
    double* g = (double*)malloc(bytes);
    double* gn = (double*)malloc(bytes);
    double* xn = (double*)malloc(bytes);
    double* d = (double*)malloc(bytes);
    double* phi = (double*)malloc(bytes);
    double* beta = (double*)malloc(bytes);
    double hist[10];
    int nh = 0;

    proj_box(n, x, l, u, x);
    gradient(pr, inv_tau, x, rhs, g);
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) f += 0.5 * x[i] * (g[i] - rhs[i]);
    hist[nh++] = f;
    double alpha = 1.0 / (norm_Q + inv_tau);
    grad_split(n, x, g, l, u, 1.0, phi, beta, NULL);
    double res = sqrt(dot(n, phi, phi) + dot(n, beta, beta));
    int64_t it = 0;
    while (res > eps && it < max_inner) {
        ++it;
        for (int64_t i = 0; i < n; ++i) d[i] = clampd(x[i] - alpha * g[i], l[i], u[i]) - x[i];
        double gd = dot(n, g, d);
        double fmax = hist[0];
        for (int h = 1; h < nh; ++h) if (hist[h] > fmax) fmax = hist[h];
        double lam = 1.0, fn = 0.0;
        for (int ls = 0; ls < 40; ++ls) {
            for (int64_t i = 0; i < n; ++i) xn[i] = x[i] + lam * d[i];
            gradient(pr, inv_tau, xn, rhs, gn);
            fn = 0.0;
            for (int64_t i = 0; i < n; ++i) fn += 0.5 * xn[i] * (gn[i] - rhs[i]);
            if (fn <= fmax + 1e-4 * lam * gd) break;
            lam *= 0.5;
        }
        double ss = 0.0, sy = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double s = xn[i] - x[i], yv = gn[i] - g[i];
            ss += s * s; sy += s * yv;
        }
        alpha = sy > 0.0 ? ss / sy : 1.0 / (norm_Q + inv_tau);
        if (alpha < 1e-12) alpha = 1e-12;
        if (alpha > 1e12) alpha = 1e12;
        memcpy(x, xn, bytes);
        memcpy(g, gn, bytes);
        if (nh < 10) hist[nh++] = fn;
        else { memmove(hist, hist + 1, sizeof(double) * 9); hist[9] = fn; }
        grad_split(n, x, g, l, u, 1.0, phi, beta, NULL);
        res = sqrt(dot(n, phi, phi) + dot(n, beta, beta));
    }
    if (res_out) *res_out = res;
    free(g); free(gn); free(xn); free(d); free(phi); free(beta);
    return it;
}

static int64_t solve_subproblem(const oprob* pr, int solver, double inv_tau, const double* rhs,
                                double* x, double eps, int64_t max_inner, double norm_Q,
                                const oracle_params* prm, double* res)
{
    if (solver == ORACLE_INNER_AUTO)
        solver = pr->qkind == QK_GENERAL ? ORACLE_INNER_MPRGP : ORACLE_INNER_CLOSED;
    if (solver == ORACLE_INNER_CLOSED) {
        closed_form(pr, inv_tau, rhs, x);
        if (res) *res = 0.0;
        return 0;
    }
    if (solver == ORACLE_INNER_BB)
        return bbpg(pr, inv_tau, rhs, x, eps, max_inner, norm_Q, res);
    double abar = prm->mprgp_abar_scale / (norm_Q + inv_tau);
    return mprgp(pr, inv_tau, rhs, x, eps, max_inner, prm->mprgp_gamma, abar, res);
}

int64_t oracle_subproblem(int64_t n,
                          const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                          const double* lv, const double* uv, double tau,
                          const double* rhs, double* x, double eps, int64_t max_inner,
                          int solver, double norm_Q, double* final_res)
{
    oracle_params prm;
    oracle_params_default(&prm);
    int64_t zero = 0;
    oprob pr;
    setup_problem(&pr, n, 0, Q_rowptr, Q_col, Q_val, &zero, NULL, NULL,
                  NULL, NULL, NULL, lv, uv);
    if (solver == ORACLE_INNER_CLOSED && pr.qkind == QK_GENERAL) { free_problem(&pr); return -1; }
    int64_t it = solve_subproblem(&pr, solver, 1.0 / tau, rhs, x, eps, max_inner, norm_Q,
                                  &prm, final_res);
    free_problem(&pr);
    return it;
}

/* ------------------------------------------------------------------------ */
/* KKT residuals (Section 4)                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double r_primal, r_dual, r_gap, pobj, dobj, natural, pviol;
} kkt_t;

static kkt_t kkt_eval(const oprob* pr, const double* x, const double* y)
{
    int64_t n = pr->n, m = pr->m;
    double* ax = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* ps = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* qx = (double*)malloc(sizeof(double) * (size_t)n);
    double* aty = (double*)malloc(sizeof(double) * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    double* rh = (double*)malloc(sizeof(double) * (size_t)n);
    double* nr = (double*)malloc(sizeof(double) * (size_t)n);
    kkt_t k;

    /* primal: ||Ax - proj_S(Ax)||_inf / (1 + max(||lc||, ||uc||)) */
    amul(pr, x, ax);
    for (int64_t i = 0; i < m; ++i) ps[i] = ax[i] - clampd(ax[i], pr->lc[i], pr->uc[i]);
    k.pviol = amax(m, ps);
    double bl = amax_finite(m, pr->lc), bu = amax_finite(m, pr->uc);
    k.r_primal = k.pviol / (1.0 + (bl > bu ? bl : bu));

    /* dual: r = Qx + c + A'y;  ||r - proj_R(r)||_inf / (1 + max(||Qx||, ||A'y||, ||c||)) */
    qmul(pr, x, qx);
    atmul(pr, y, aty);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = qx[i] + pr->c[i] + aty[i];
        rh[i] = proj_R1(r[i], pr->lv[i], pr->uv[i]);
        nr[i] = r[i] - rh[i];
    }
    double dviol = amax(n, nr);
    double s1 = amax(n, qx), s2 = amax(n, aty), s3 = amax(n, pr->c);
    double sd = s1 > s2 ? s1 : s2;
    sd = sd > s3 ? sd : s3;
    k.r_dual = dviol / (1.0 + sd);

    /* gap: x'Qx + c'x + p(-rhat; lv, uv) + p(y; lc, uc) */
    double xqx = dot(n, x, qx), cx = dot(n, pr->c, x);
    for (int64_t i = 0; i < n; ++i) nr[i] = -rh[i];
    double pr_ = oracle_support(n, nr, pr->lv, pr->uv);
    double py = oracle_support(m, y, pr->lc, pr->uc);
    k.pobj = 0.5 * xqx + cx;
    k.dobj = -pr_ - 0.5 * xqx - py;
    double gap = fabs(xqx + cx + pr_ + py);
    double d1 = fabs(k.pobj), d2 = fabs(0.5 * xqx + pr_ + py);
    k.r_gap = gap / (1.0 + (d1 > d2 ? d1 : d2));

    /* natural residual ||x - proj_X(x - r)||_inf (diagnostic) */
    for (int64_t i = 0; i < n; ++i) nr[i] = x[i] - clampd(x[i] - r[i], pr->lv[i], pr->uv[i]);
    k.natural = amax(n, nr);

    free(ax); free(ps); free(qx); free(aty); free(r); free(rh); free(nr);
    return k;
}

void oracle_kkt(int64_t n, int64_t m,
                const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                const double* c, const double* lc, const double* uc,
                const double* lv, const double* uv,
                const double* x, const double* y, double* out)
{
    oprob pr;
    setup_problem(&pr, n, m, Q_rowptr, Q_col, Q_val, A_rowptr, A_col, A_val, c, lc, uc, lv, uv);
    kkt_t k = kkt_eval(&pr, x, y);
    out[0] = k.r_primal; out[1] = k.r_dual; out[2] = k.r_gap;
    out[3] = k.pobj; out[4] = k.dobj; out[5] = k.natural; out[6] = k.pviol;
    free_problem(&pr);
}

/* ------------------------------------------------------------------------ */
/* infeasibility certificates (Section 5)                                    */
/* ------------------------------------------------------------------------ */

/* sum of |u_i| z_i^+ + |l_i| z_i^- (magnitudes of the terms of p) */
static double support_abs(int64_t k, const double* z, const double* l, const double* u)
{
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        if (z[i] > 0.0) s += fabs(u[i]) * z[i];
        else if (z[i] < 0.0) s += fabs(l[i]) * (-z[i]);
    }
    return s;
}

/* Primal infeasibility: ytil = proj_Y(dy); fires when the dual objective of
 * the feasibility problem improves along ytil, I = [p(-proj_R(A'ytil)) +
 * p(ytil)]^- > 1e-9 * (sum of the magnitudes of the terms of both p), and
 * ||A'ytil - proj_R(A'ytil)||_inf <= eps_inf * I. */
static int primal_infeasible(const oprob* pr, const double* dy, double eps_inf, double* ray)
{
    int64_t n = pr->n, m = pr->m;
    if (m == 0) return 0;
    double* yt = (double*)malloc(sizeof(double) * (size_t)m);
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* wh = (double*)malloc(sizeof(double) * (size_t)n);
    double* dv = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < m; ++i) yt[i] = proj_Y1(dy[i], pr->lc[i], pr->uc[i]);
    double ny = amax(m, yt);
    int fire = 0;
    if (ny > 0.0 && isfinite(ny)) {
        atmul(pr, yt, w);
        for (int64_t i = 0; i < n; ++i) {
            wh[i] = proj_R1(w[i], pr->lv[i], pr->uv[i]);
            dv[i] = w[i] - wh[i];
        }
        double viol = amax(n, dv);
        for (int64_t i = 0; i < n; ++i) dv[i] = -wh[i];
        double val = oracle_support(n, dv, pr->lv, pr->uv) + oracle_support(m, yt, pr->lc, pr->uc);
        double imp = val < 0.0 ? -val : 0.0;
        /* the improvement must stand out of the rounding of the sums that
         * produced it: compare with the sum of the terms' magnitudes */
        double mag = support_abs(n, dv, pr->lv, pr->uv) + support_abs(m, yt, pr->lc, pr->uc);
        fire = imp > 1e-9 * mag && viol <= eps_inf * imp;
        if (ray) for (int64_t i = 0; i < m; ++i) ray[i] = yt[i] / ny;
    } else if (ray) {
        for (int64_t i = 0; i < m; ++i) ray[i] = 0.0;
    }
    free(yt); free(w); free(wh); free(dv);
    return fire;
}

/* Dual infeasibility: d = proj_{Recc X}(dx), dtil = d/||d||_inf; fires when
 * c'dtil < -eps_tol and max(||A dtil - proj_{Recc S}(A dtil)||_inf,
 * ||Q dtil||_inf / gamma_Q) <= eps_inf, gamma_Q = max(1, max_i sum_j |Q_ij|). */
static int dual_infeasible(const oprob* pr, const double* dx, double eps_tol, double eps_inf,
                           double* ray)
{
    int64_t n = pr->n, m = pr->m;
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    double* qd = (double*)malloc(sizeof(double) * (size_t)n);
    double* ad = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    for (int64_t i = 0; i < n; ++i) d[i] = proj_rec1(dx[i], pr->lv[i], pr->uv[i]);
    double nd = amax(n, d);
    int fire = 0;
    if (nd > 0.0 && isfinite(nd)) {
        for (int64_t i = 0; i < n; ++i) d[i] /= nd;
        double cd = dot(n, pr->c, d);
        if (cd < -eps_tol) {
            amul(pr, d, ad);
            for (int64_t i = 0; i < m; ++i) ad[i] -= proj_rec1(ad[i], pr->lc[i], pr->uc[i]);
            double v1 = amax(m, ad);
            qmul(pr, d, qd);
            double gq = 1.0;
            if (pr->qkind == QK_GENERAL) {
                for (int64_t i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int64_t k = pr->Qp[i]; k < pr->Qp[i + 1]; ++k) s += fabs(pr->Qv[k]);
                    if (s > gq) gq = s;
                }
            } else {
                for (int64_t i = 0; i < n; ++i) if (fabs(pr->qdiag[i]) > gq) gq = fabs(pr->qdiag[i]);
            }
            double v2 = amax(n, qd) / gq;
            fire = (v1 > v2 ? v1 : v2) <= eps_inf;
        }
        if (ray) memcpy(ray, d, sizeof(double) * (size_t)n);
    } else if (ray) {
        for (int64_t i = 0; i < n; ++i) ray[i] = 0.0;
    }
    free(d); free(qd); free(ad);
    return fire;
}

int oracle_primal_infeasible(int64_t n, int64_t m,
                             const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                             const double* lc, const double* uc,
                             const double* lv, const double* uv,
                             const double* dy, double eps_inf, double* ray_out)
{
    oprob pr;
    setup_problem(&pr, n, m, NULL, NULL, NULL, A_rowptr, A_col, A_val, NULL, lc, uc, lv, uv);
    int f = primal_infeasible(&pr, dy, eps_inf, ray_out);
    free_problem(&pr);
    return f;
}

int oracle_dual_infeasible(int64_t n, int64_t m,
                           const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                           const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                           const double* c, const double* lc, const double* uc,
                           const double* lv, const double* uv,
                           const double* dx, double eps_tol, double eps_inf, double* ray_out)
{
    oprob pr;
    setup_problem(&pr, n, m, Q_rowptr, Q_col, Q_val, A_rowptr, A_col, A_val, c, lc, uc, lv, uv);
    int f = dual_infeasible(&pr, dx, eps_tol, eps_inf, ray_out);
    free_problem(&pr);
    return f;
}

/* ------------------------------------------------------------------------ */
/* the solver                                                                */
/* ------------------------------------------------------------------------ */

/* Reflected Halpern step (Section 3.1, reading of the garbled display):
 * z+ = ((t+1)/(t+2)) ((1+theta) T(z) - theta z) + z_anchor/(t+2), with t
 * counting iterations since the last restart and z_anchor the restart point.
 * out may alias z. */
void oracle_halpern(int64_t k, int64_t t, double theta, const double* zt, const double* z,
                    const double* za, double* out)
{
    double w = (double)(t + 1) / (double)(t + 2), wa = 1.0 / (double)(t + 2);
    for (int64_t i = 0; i < k; ++i)
        out[i] = w * ((1.0 + theta) * zt[i] - theta * z[i]) + wa * za[i];
}

/* PID update of the primal weight at the end of a restart round (Section
 * 3.2, eq. pid): e = log(sqrt(omega) mx / (my / sqrt(omega))) with mx, my
 * the primal and dual movement over the round; log omega decreases by
 * kp e + ki (sum of e) + kd (e - e_prev).  Skipped when a movement is below
 * 1e-10; log omega is kept within log(omega0) +- 10. */
double oracle_pid(double omega, double omega0, double mx, double my, double kp, double ki,
                  double kd, double* integral, double* prev_e)
{
    if (!(mx > 1e-10 && my > 1e-10 && isfinite(mx) && isfinite(my))) return omega;
    double e = log(sqrt(omega) * mx / (my / sqrt(omega)));
    *integral += e;
    double lw = log(omega) - (kp * e + ki * (*integral) + kd * (e - *prev_e));
    *prev_e = e;
    return exp(clampd(lw, log(omega0) - 10.0, log(omega0) + 10.0));
}

/* Adaptive inner tolerance (Section 3.3):
 * eps_k = min(eps_{k-1}, max(gamma * omega * ||x_k - x_{k-1}|| / tau, eps_min)). */
double oracle_inner_tol(double eps_prev, double gamma, double omega, double tau, double move,
                        double eps_min)
{
    return fmin(eps_prev, fmax(gamma * omega * move / tau, eps_min));
}

/* Restart test (reading; the paper names restart rounds but gives no rule):
 * restart when R <= sufficient * R_start, or R <= necessary * R_start while
 * R grew since the previous check of the round, or when the round has run
 * t >= artificial * k iterations. */
int oracle_restart_test(double R, double R_start, double R_prev, int R_prev_valid, int64_t t,
                        int64_t k, const oracle_params* p)
{
    return R <= p->restart_sufficient * R_start
        || (R_prev_valid && R <= p->restart_necessary * R_start && R > R_prev)
        || (double)t >= p->restart_artificial * (double)k;
}

static int has_nonfinite(int64_t k, const double* v)
{
    for (int64_t i = 0; i < k; ++i) if (!isfinite(v[i])) return 1;
    return 0;
}

int oracle_qp_solve(int64_t n, int64_t m,
                    const int64_t* Qp, const int32_t* Qj, const double* Qv,
                    const int64_t* Ap, const int32_t* Aj, const double* Av,
                    const double* c, const double* lc, const double* uc,
                    const double* lv, const double* uv,
                    const oracle_params* prm_in,
                    double* x_out, double* y_out, oracle_info* info)
{
    oracle_params prm;
    if (prm_in) prm = *prm_in; else oracle_params_default(&prm);
    if (n < 1 || m < 0 || !Ap || !c || !lv || !uv || (m > 0 && (!lc || !uc))) return -1;
    for (int64_t i = 0; i < n; ++i) if (lv[i] > uv[i]) return -1;
    for (int64_t i = 0; i < m; ++i) if (lc[i] > uc[i]) return -1;

    const double t_call = wall_seconds();
    oprob pr;
    setup_problem(&pr, n, m, Qp, Qj, Qv, Ap, Aj, Av, c, lc, uc, lv, uv);
    oracle_info inf;
    memset(&inf, 0, sizeof(inf));

    /* step sizes: eta = 0.998 / ||A||_2 (Section 3.2), ||A|| by power iteration */
    double normA = oracle_norm2(m, n, Ap, Aj, Av, prm.power_tol, prm.power_max_iter, NULL);
    double eta = normA * prm.norm_safety > 1e-12 ? prm.eta_scale / (prm.norm_safety * normA) : 1.0;
    double normQ = 0.0;
    if (pr.qkind == QK_GENERAL)
        normQ = prm.norm_safety * oracle_norm2(n, n, Qp, Qj, Qv, prm.power_tol, prm.power_max_iter, NULL);
    else
        for (int64_t i = 0; i < n; ++i) if (fabs(pr.qdiag[i]) > normQ) normQ = fabs(pr.qdiag[i]);

    /* initial primal weight ||c||_2 / ||btil||_2, btil_i the finite bound of row i */
    double nb = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double bt = isfinite(lc[i]) ? lc[i] : (isfinite(uc[i]) ? uc[i] : 0.0);
        nb += bt * bt;
    }
    nb = sqrt(nb);
    double nc = nrm2(n, c);
    double omega0 = (nc > 1e-10 && nb > 1e-10) ? nc / nb : 1.0;
    double omega = omega0;

    size_t bn = sizeof(double) * (size_t)n, bm = sizeof(double) * (size_t)(m + 1);
    double* x = (double*)malloc(bn);    /* z^k, primal */
    double* y = (double*)calloc((size_t)(m + 1), sizeof(double));
    double* xa = (double*)malloc(bn);   /* anchor z^{n,0} */
    double* ya = (double*)malloc(bm);
    double* xt = (double*)malloc(bn);   /* T(z^k) */
    double* yt = (double*)malloc(bm);
    double* rhs = (double*)malloc(bn);
    double* aty = (double*)malloc(bn);
    double* xb = (double*)malloc(bn);
    double* axb = (double*)malloc(bm);
    double* dx = (double*)malloc(bn);
    double* dy = (double*)malloc(bm);
    double* dxr = (double*)malloc(bn);
    double* dyr = (double*)malloc(bm);

    /* start: x0 = proj_X(0), y0 = 0 */
    for (int64_t i = 0; i < n; ++i) x[i] = clampd(0.0, lv[i], uv[i]);
    memcpy(xa, x, bn); memcpy(xt, x, bn);
    memcpy(ya, y, bm); memcpy(yt, y, bm);
    memset(dx, 0, bn); memset(dy, 0, bm);

    double eps = INFINITY;
    double pid_int = 0.0, pid_prev = 0.0;
    double R_start = 0.0, R_prev = 0.0;
    int R_prev_valid = 0;
    int64_t k = 0, t = 0;
    int status = ORACLE_NOT_SOLVED;
    kkt_t kk;
    memset(&kk, 0, sizeof(kk));
    inf.seconds_setup = wall_seconds() - t_call;
    double check_t0 = -1.0;   /* start of the check in progress, if any */

    for (;;) {
        if (k > 0 || prm.max_iter == 0) {
            /* ---------------- check ------------------------------------ */
            if (k % prm.check_every == 0 || k >= prm.max_iter) {
                check_t0 = wall_seconds();
                inf.checks++;
                kk = kkt_eval(&pr, xt, yt);
                double worst = fmax(kk.r_primal, fmax(kk.r_dual, kk.r_gap));
                if (prm.verbose)
                    fprintf(stderr, "[oracle] k=%lld t=%lld rp=%.3e rd=%.3e rg=%.3e omega=%.4e "
                            "eps=%.3e inner=%lld restarts=%lld\n", (long long)k, (long long)t,
                            kk.r_primal, kk.r_dual, kk.r_gap, omega, eps,
                            (long long)inf.inner_iterations, (long long)inf.restarts);
                if (worst != worst || has_nonfinite(n, xt) || has_nonfinite(m, yt)) {
                    status = ORACLE_NUMERICAL_ERROR;
                    break;
                }
                if (worst <= prm.tol) { status = ORACLE_OPTIMAL; break; }
                if (k > 0 && primal_infeasible(&pr, dy, prm.eps_inf, y_out)) {
                    status = ORACLE_PRIMAL_INFEASIBLE;
                    break;
                }
                if (k > 0 && dual_infeasible(&pr, dx, prm.tol, prm.eps_inf, x_out)) {
                    status = ORACLE_DUAL_INFEASIBLE;
                    break;
                }
                if (k >= prm.max_iter) { status = ORACLE_ITERATION_LIMIT; break; }

                /* restart test on the weighted fixed-point residual */
                double R = sqrt(omega * dot(n, dx, dx) + dot(m, dy, dy) / omega);
                int restart = oracle_restart_test(R, R_start, R_prev, R_prev_valid, t, k, &prm);
                R_prev = R; R_prev_valid = 1;
                if (restart) {
                    /* PID on log(omega) over the round (Section 3.2, eq. pid) */
                    for (int64_t i = 0; i < n; ++i) dxr[i] = xt[i] - xa[i];
                    for (int64_t i = 0; i < m; ++i) dyr[i] = yt[i] - ya[i];
                    double mx = nrm2(n, dxr), my = nrm2(m, dyr);
                    omega = oracle_pid(omega, omega0, mx, my, prm.kp, prm.ki, prm.kd,
                                       &pid_int, &pid_prev);
                    memcpy(xa, xt, bn); memcpy(ya, yt, bm);
                    memcpy(x, xt, bn); memcpy(y, yt, bm);
                    t = 0;
                    R_prev_valid = 0;
                    inf.restarts++;
                }
                inf.seconds_check += wall_seconds() - check_t0;
                check_t0 = -1.0;
            }
        }
        if (k >= prm.max_iter) { status = ORACLE_ITERATION_LIMIT; break; }

        double tau = eta / omega, sigma = eta * omega, inv_tau = 1.0 / tau;

        /* ---------------- primal step (eq. primal_update) ------------------ */
        atmul(&pr, y, aty);
        for (int64_t i = 0; i < n; ++i) rhs[i] = x[i] * inv_tau - c[i] - aty[i];
        /* warm start at the previous T(z) (already in xt) */
        if (isinf(eps) && prm.eps_inner_fixed <= 0.0 && pr.qkind == QK_GENERAL) {
            double r0 = proj_grad_norm(&pr, inv_tau, xt, rhs);
            eps = fmax(prm.gamma_inner * r0, prm.eps_min);
        }
        double eps_use = prm.eps_inner_fixed > 0.0 ? prm.eps_inner_fixed : eps;
        const double t_inner = wall_seconds();
        inf.inner_iterations += solve_subproblem(&pr, prm.inner_solver, inv_tau, rhs, xt,
                                                 eps_use, prm.max_inner, normQ, &prm, NULL);
        inf.seconds_inner += wall_seconds() - t_inner;

        /* ---------------- dual step (eq. extrapolation, dual_update) -------- */
        for (int64_t i = 0; i < n; ++i) xb[i] = 2.0 * xt[i] - x[i];
        amul(&pr, xb, axb);
        for (int64_t i = 0; i < m; ++i) {
            double v = y[i] / sigma + axb[i];
            yt[i] = sigma * (v - clampd(v, lc[i], uc[i]));
        }

        /* ---------------- movement and Halpern averaging (Section 3.1) ----- */
        for (int64_t i = 0; i < n; ++i) dx[i] = xt[i] - x[i];
        for (int64_t i = 0; i < m; ++i) dy[i] = yt[i] - y[i];
        double ndx = nrm2(n, dx), ndy = nrm2(m, dy);
        if (prm.use_halpern) {
            oracle_halpern(n, t, prm.theta, xt, x, xa, x);
            oracle_halpern(m, t, prm.theta, yt, y, ya, y);
        } else {
            memcpy(x, xt, bn); memcpy(y, yt, bm);
        }

        /* ---------------- adaptive inner tolerance (Section 3.3) ----------- */
        if (prm.eps_inner_fixed <= 0.0)
            eps = oracle_inner_tol(eps, prm.gamma_inner, omega, tau, ndx, prm.eps_min);

        ++k; ++t;
        if (t == 1) R_start = sqrt(omega * ndx * ndx + ndy * ndy / omega);
    }

    if (check_t0 >= 0.0) inf.seconds_check += wall_seconds() - check_t0;
    inf.status = status;
    inf.iterations = k;
    inf.r_primal = kk.r_primal; inf.r_dual = kk.r_dual; inf.r_gap = kk.r_gap;
    inf.primal_obj = kk.pobj; inf.dual_obj = kk.dobj;
    inf.natural_residual = kk.natural;
    inf.omega = omega; inf.eta = eta; inf.norm_A = normA; inf.norm_Q = normQ;
    inf.eps_inner = eps;
    if (status != ORACLE_PRIMAL_INFEASIBLE && status != ORACLE_DUAL_INFEASIBLE) {
        if (x_out) memcpy(x_out, xt, bn);
        if (y_out && m > 0) memcpy(y_out, yt, sizeof(double) * (size_t)m);
    } else if (status == ORACLE_PRIMAL_INFEASIBLE) {
        if (x_out) memcpy(x_out, xt, bn);
    } else {
        if (y_out && m > 0) memcpy(y_out, yt, sizeof(double) * (size_t)m);
    }
    if (info) *info = inf;

    free(x); free(y); free(xa); free(ya); free(xt); free(yt); free(rhs); free(aty);
    free(xb); free(axb); free(dx); free(dy); free(dxr); free(dyr);
    free_problem(&pr);
    if (info) info->seconds_total = wall_seconds() - t_call;
    return status;
}
