/* Drives every entry point of the CPU oracle on small problems, for the
 * AddressSanitizer / UndefinedBehaviorSanitizer build of
 * tests/test_sanitizers.py: boxed and unboxed QPs, an LP, a problem without
 * rows, a primal-infeasible and an unbounded problem, the subproblem
 * solvers, the norm estimate and the certificate tests.  Exits non-zero if a
 * status differs from the one the problem is built to have. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pdhcg_oracle.h"

static unsigned long long lcg_state = 88172645463325252ull;
static double urand(void) /* U(0, 1) from a 64-bit LCG (Knuth's MMIX constants) */
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
    int64_t rows, cols;
    int64_t* rp;
    int32_t* cj;
    double* v;
} csr;

static csr dense_to_csr(int64_t r, int64_t c, const double* d)
{
    csr M = {r, c, calloc((size_t)r + 1, sizeof(int64_t)), NULL, NULL};
    int64_t nnz = 0;
    for (int64_t i = 0; i < r * c; ++i) nnz += d[i] != 0.0;
    M.cj = malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    M.v = malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < r; ++i) {
        for (int64_t j = 0; j < c; ++j)
            if (d[i * c + j] != 0.0) { M.cj[k] = (int32_t)j; M.v[k] = d[i * c + j]; ++k; }
        M.rp[i + 1] = k;
    }
    return M;
}

static void free_csr(csr* M) { free(M->rp); free(M->cj); free(M->v); }

static int check(const char* what, int got, int want)
{
    printf("%-28s status %d (want %d)\n", what, got, want);
    return got == want ? 0 : 1;
}

int main(void)
{
    int bad = 0;
    const int64_t n = 40, m = 16;
    double* Bd = calloc((size_t)(n * n), sizeof(double));
    double* Qd = calloc((size_t)(n * n), sizeof(double));
    double* Ad = calloc((size_t)(m * n), sizeof(double));
    for (int64_t i = 0; i < n / 2; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (urand() < 0.2) Bd[i * n + j] = 2.0 * urand() - 1.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = i == j ? 0.1 : 0.0;
            for (int64_t r = 0; r < n / 2; ++r) s += Bd[r * n + i] * Bd[r * n + j];
            Qd[i * n + j] = s;
        }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (urand() < 0.25) Ad[i * n + j] = 2.0 * urand() - 1.0;
    csr Q = dense_to_csr(n, n, Qd), A = dense_to_csr(m, n, Ad);
    double *c = malloc(sizeof(double) * n), *x0 = malloc(sizeof(double) * n);
    double *lv = malloc(sizeof(double) * n), *uv = malloc(sizeof(double) * n);
    double *b = malloc(sizeof(double) * m), *lc = malloc(sizeof(double) * m), *uc = malloc(sizeof(double) * m);
    char* sense = malloc((size_t)m);
    for (int64_t j = 0; j < n; ++j) {
        c[j] = 2.0 * urand() - 1.0;
        x0[j] = urand() - 0.5;
        lv[j] = -1.0;
        uv[j] = 1.0;
    }
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += Ad[i * n + j] * x0[j];
        sense[i] = i < m / 2 ? 'E' : 'G';
        b[i] = i < m / 2 ? s : s - 0.05;
    }
    if (oracle_bounds_from_sense(m, b, sense, lc, uc) != 0) bad++;

    oracle_params p;
    oracle_params_default(&p);
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * (m + 1));
    oracle_info info;
    double kkt[7];

    /* boxed QP (MPRGP inner solve), then BB, then unboxed */
    bad += check("boxed QP, MPRGP", oracle_qp_solve(n, m, Q.rp, Q.cj, Q.v, A.rp, A.cj, A.v, c, lc, uc, lv, uv,
                                                    &p, x, y, &info), ORACLE_OPTIMAL);
    oracle_kkt(n, m, Q.rp, Q.cj, Q.v, A.rp, A.cj, A.v, c, lc, uc, lv, uv, x, y, kkt);
    if (!(fmax(kkt[0], fmax(kkt[1], kkt[2])) <= 1e-6)) bad++;
    p.inner_solver = ORACLE_INNER_BB;
    bad += check("boxed QP, BB", oracle_qp_solve(n, m, Q.rp, Q.cj, Q.v, A.rp, A.cj, A.v, c, lc, uc, lv, uv,
                                                 &p, x, y, &info), ORACLE_OPTIMAL);
    p.inner_solver = ORACLE_INNER_AUTO;
    double *lfree = malloc(sizeof(double) * n), *ufree = malloc(sizeof(double) * n);
    for (int64_t j = 0; j < n; ++j) { lfree[j] = -INFINITY; ufree[j] = INFINITY; }
    bad += check("unboxed QP, CG", oracle_qp_solve(n, m, Q.rp, Q.cj, Q.v, A.rp, A.cj, A.v, c, lc, uc, lfree,
                                                   ufree, &p, x, y, &info), ORACLE_OPTIMAL);
    /* LP (Q = 0) and a problem without rows */
    bad += check("boxed LP", oracle_qp_solve(n, m, NULL, NULL, NULL, A.rp, A.cj, A.v, c, lc, uc, lv, uv, &p, x,
                                             y, &info), ORACLE_OPTIMAL);
    int64_t rp0[1] = {0};
    bad += check("no rows", oracle_qp_solve(n, 0, Q.rp, Q.cj, Q.v, rp0, NULL, NULL, c, NULL, NULL, lv, uv, &p,
                                            x, y, &info), ORACLE_OPTIMAL);
    /* iteration limit 0: the start point's residuals */
    p.max_iter = 0;
    bad += check("max_iter = 0", oracle_qp_solve(n, m, Q.rp, Q.cj, Q.v, A.rp, A.cj, A.v, c, lc, uc, lv, uv,
                                                 &p, x, y, &info), ORACLE_ITERATION_LIMIT);
    p.max_iter = 100000;

    /* primal infeasible: row 1 := row 0 with b shifted */
    double* Ad2 = malloc(sizeof(double) * (size_t)(m * n));
    memcpy(Ad2, Ad, sizeof(double) * (size_t)(m * n));
    memcpy(Ad2 + n, Ad2, sizeof(double) * (size_t)n);
    csr A2 = dense_to_csr(m, n, Ad2);
    double *lc2 = malloc(sizeof(double) * m), *uc2 = malloc(sizeof(double) * m);
    memcpy(lc2, lc, sizeof(double) * m);
    memcpy(uc2, uc, sizeof(double) * m);
    lc2[1] = uc2[1] = lc[0] + 1.0;
    lc2[0] = uc2[0] = lc[0];
    p.max_iter = 20000;
    bad += check("contradictory rows", oracle_qp_solve(n, m, Q.rp, Q.cj, Q.v, A2.rp, A2.cj, A2.v, c, lc2, uc2,
                                                       lfree, ufree, &p, x, y, &info), ORACLE_PRIMAL_INFEASIBLE);
    /* unbounded: variable 0 free below, untouched by rows and Q, cost 1 */
    double* Ad3 = malloc(sizeof(double) * (size_t)(m * n));
    memcpy(Ad3, Ad, sizeof(double) * (size_t)(m * n));
    for (int64_t i = 0; i < m; ++i) Ad3[i * n] = 0.0;
    csr A3 = dense_to_csr(m, n, Ad3);
    double *lv3 = malloc(sizeof(double) * n), *c3 = malloc(sizeof(double) * n);
    memcpy(lv3, lv, sizeof(double) * n);
    memcpy(c3, c, sizeof(double) * n);
    lv3[0] = -INFINITY;
    c3[0] = 1.0;
    double* lc3 = malloc(sizeof(double) * m), *uc3 = malloc(sizeof(double) * m);
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += Ad3[i * n + j] * x0[j];
        lc3[i] = s - 0.05;
        uc3[i] = INFINITY;
    }
    bad += check("unbounded LP", oracle_qp_solve(n, m, NULL, NULL, NULL, A3.rp, A3.cj, A3.v, c3, lc3, uc3, lv3,
                                                 uv, &p, x, y, &info), ORACLE_DUAL_INFEASIBLE);
    p.max_iter = 100000;

    /* the pieces on their own */
    double *rhs = malloc(sizeof(double) * n), res = 0.0;
    for (int64_t j = 0; j < n; ++j) rhs[j] = 3.0 * c[j];
    for (int solver = ORACLE_INNER_MPRGP; solver <= ORACLE_INNER_BB; ++solver) {
        memset(x, 0, sizeof(double) * n);
        oracle_subproblem(n, Q.rp, Q.cj, Q.v, lv, uv, 0.5, rhs, x, 1e-10, 5000, solver, 40.0, &res);
        if (!(res <= 1e-10)) bad++;
    }
    int64_t it = 0;
    const double na = oracle_norm2(m, n, A.rp, A.cj, A.v, 1e-7, 1000, &it);
    if (!(na > 0.0)) bad++;
    double* z = malloc(sizeof(double) * n);
    for (int64_t j = 0; j < n; ++j) z[j] = urand() - 0.5;
    (void)oracle_support(n, z, lfree, ufree);
    (void)oracle_support(n, z, lv, uv);
    double* ray = malloc(sizeof(double) * (n + m + 1));
    (void)oracle_primal_infeasible(n, m, A.rp, A.cj, A.v, lc, uc, lv, uv, z, 1e-8, ray);
    (void)oracle_dual_infeasible(n, m, Q.rp, Q.cj, Q.v, A.rp, A.cj, A.v, c, lc, uc, lv3, uv, z, 1e-6, 1e-8, ray);
    double hz[4];
    oracle_halpern(4, 3, 1.0, z, z + 4, z + 8, hz);
    double integ = 0.0, prev = 0.0;
    (void)oracle_pid(1.0, 1.0, 0.5, 2.0, 0.99, 0.01, 0.0, &integ, &prev);
    (void)oracle_inner_tol(INFINITY, 5e-4, 1.0, 0.3, 1e-3, 1e-9);
    (void)oracle_restart_test(0.1, 1.0, 0.2, 1, 10, 100, &p);
    (void)oracle_splitmix_unit(12345);

    free_csr(&Q); free_csr(&A); free_csr(&A2); free_csr(&A3);
    free(Bd); free(Qd); free(Ad); free(Ad2); free(Ad3);
    free(c); free(x0); free(lv); free(uv); free(b); free(lc); free(uc); free(sense); free(x); free(y);
    free(lfree); free(ufree); free(lc2); free(uc2); free(lv3); free(c3); free(lc3); free(uc3);
    free(rhs); free(z); free(ray);
    printf("oracle driver: %d failure(s)\n", bad);
    return bad ? 1 : 0;
}
