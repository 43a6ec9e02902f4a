/*
 * pdhcg_oracle.h -- plain FP64 CPU reference of PDHCG-II for convex QP.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source, header, helper or
 * constant table with the HIP path.
 *
 * Problem (Section 2, eq. QP):  min 1/2 x'Qx + c'x  s.t.  lc <= Ax <= uc,
 * lv <= x <= uv, with Q symmetric PSD given as full CSR (both triangles).
 * Bounds may be +-INFINITY.
 *
 * Parity status of each piece is stated in pdhcg_oracle.c's header.
 */
#ifndef PDHCG_ORACLE_H
#define PDHCG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_NOT_SOLVED = 0,
    ORACLE_OPTIMAL = 1,
    ORACLE_PRIMAL_INFEASIBLE = 2,
    ORACLE_DUAL_INFEASIBLE = 3,
    ORACLE_ITERATION_LIMIT = 4,
    ORACLE_NUMERICAL_ERROR = 5
};

/* inner solver choice for the primal subproblem (Section 2.2) */
enum {
    ORACLE_INNER_AUTO = 0,   /* closed form if Q diagonal, else MPRGP (CG when unboxed) */
    ORACLE_INNER_MPRGP = 1,  /* CG on the free set with expansion / proportioning */
    ORACLE_INNER_BB = 2,     /* projected gradient with Barzilai-Borwein steps */
    ORACLE_INNER_CLOSED = 3  /* closed form; only valid when Q is diagonal or absent */
};

typedef struct {
    double tol;              /* eps_tol on max(r_primal, r_dual, r_gap) */
    int64_t max_iter;        /* outer PDHG iterations */
    int64_t check_every;     /* KKT / infeasibility / restart cadence */
    int64_t max_inner;       /* cap on inner iterations per subproblem */
    int inner_solver;        /* ORACLE_INNER_* */
    int use_halpern;         /* 1: reflected Halpern averaging, 0: plain PDHG */
    double theta;            /* reflection parameter */
    double kp, ki, kd;       /* PID gains on log(omega) */
    double gamma_inner;      /* adaptive inner tolerance factor (5e-4) */
    double eps_min;          /* inner tolerance floor (1e-9) */
    double eps_inner_fixed;  /* > 0: use this fixed inner tolerance instead */
    double restart_sufficient, restart_necessary, restart_artificial;
    double eps_inf;          /* infeasibility certificate tolerance */
    double eta_scale;        /* eta = eta_scale / (norm_safety * ||A||_2) */
    double norm_safety;
    double power_tol;        /* power iteration relative-change tolerance */
    int64_t power_max_iter;
    double mprgp_gamma;      /* MPRGP proportioning constant */
    double mprgp_abar_scale; /* MPRGP expansion step abar = scale / ||H||_2 */
    int verbose;             /* print one line per check to stderr */
} oracle_params;

typedef struct {
    int status;
    int64_t iterations;
    int64_t inner_iterations;
    int64_t restarts;
    int64_t checks;
    double r_primal, r_dual, r_gap;
    double primal_obj, dual_obj;
    double omega, eta, norm_A, norm_Q;
    double eps_inner;        /* final inner tolerance */
    double natural_residual; /* ||x - proj_X(x - r)||_inf at the returned point */
    /* wall-clock seconds (instrumentation for the CPU baseline; no effect on
     * any result): setup (norm estimates), the inner subproblem solves, the
     * checks (KKT, certificates, restart), and the whole call */
    double seconds_setup, seconds_inner, seconds_check, seconds_total;
} oracle_info;

void oracle_params_default(oracle_params* p);

/* 'E' -> [b, b], 'G' -> [b, +inf), 'L' -> (-inf, b].  Returns 0 or -1 on an
 * unknown sense character. */
int oracle_bounds_from_sense(int64_t m, const double* b, const char* sense,
                             double* lc, double* uc);

/* Full solve.  Q_rowptr == NULL means Q = 0.  x_out (n) and y_out (m) may be
 * NULL.  On PRIMAL_INFEASIBLE y_out holds the ray normalised to
 * ||y||_inf = 1; on DUAL_INFEASIBLE x_out holds the ray with ||d||_inf = 1.
 * Returns the status (>= 0) or -1 on invalid input. */
int oracle_qp_solve(int64_t n, int64_t m,
                    const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                    const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                    const double* c, const double* lc, const double* uc,
                    const double* lv, const double* uv,
                    const oracle_params* prm,
                    double* x_out, double* y_out, oracle_info* info);

/* KKT residuals of Section 4 at a given (x, y).  out[0..6] = r_primal,
 * r_dual, r_gap, primal objective, dual objective, natural residual,
 * ||A x - proj_S(A x)||_inf (unnormalised). */
void oracle_kkt(int64_t n, int64_t m,
                const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                const double* c, const double* lc, const double* uc,
                const double* lv, const double* uv,
                const double* x, const double* y, double* out);

/* One primal subproblem (eq. primal_update):
 *   argmin_{lv <= x <= uv} 1/2 x'(Q + I/tau)x - rhs'x
 * x is the warm start on entry and the result on exit.  Stops when the
 * projected-gradient 2-norm is <= eps or after max_inner iterations.
 * norm_Q is ||Q||_2 (used by MPRGP's expansion step and BB's first step).
 * Returns the number of inner iterations. */
int64_t oracle_subproblem(int64_t n,
                          const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                          const double* lv, const double* uv, double tau,
                          const double* rhs, double* x, double eps, int64_t max_inner,
                          int solver, double norm_Q, double* final_res);

/* Power-iteration estimate of ||M||_2 for an (r x c) CSR matrix M (via
 * M'M), from the fixed start vector described in pdhcg_oracle.c. */
double oracle_norm2(int64_t r, int64_t c, const int64_t* rowptr, const int32_t* col,
                    const double* val, double tol, int64_t max_iter, int64_t* iters);

/* y = M x for an (r x ?) CSR matrix. */
void oracle_csr_matvec(int64_t r, const int64_t* rowptr, const int32_t* col,
                       const double* val, const double* x, double* y);

/* p(z; l, u) = u'z^+ - l'z^- with 0 * inf = 0 (Section 2, eq. dualQP). */
double oracle_support(int64_t k, const double* z, const double* l, const double* u);

/* Primal/dual infeasibility tests of Section 5 on explicit candidate rays.
 * dy (m) and dx (n) are iterate differences; returns 1 if the test fires.
 * The projected, normalised ray is written to ray_out when non-NULL. */
int oracle_primal_infeasible(int64_t n, int64_t m,
                             const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                             const double* lc, const double* uc,
                             const double* lv, const double* uv,
                             const double* dy, double eps_inf, double* ray_out);
int oracle_dual_infeasible(int64_t n, int64_t m,
                           const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                           const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                           const double* c, const double* lc, const double* uc,
                           const double* lv, const double* uv,
                           const double* dx, double eps_tol, double eps_inf, double* ray_out);

/* Pieces of the outer loop, exported so their algebra can be checked on
 * hand values.  See pdhcg_oracle.c for the reading each one takes. */
void oracle_halpern(int64_t k, int64_t t, double theta, const double* zt, const double* z,
                    const double* za, double* out);
double oracle_pid(double omega, double omega0, double mx, double my, double kp, double ki,
                  double kd, double* integral, double* prev_e);
double oracle_inner_tol(double eps_prev, double gamma, double omega, double tau, double move,
                        double eps_min);
int oracle_restart_test(double R, double R_start, double R_prev, int R_prev_valid, int64_t t,
                        int64_t k, const oracle_params* p);

/* Counter-based generator used for the power-iteration start vector:
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) applied to the counter i. */
double oracle_splitmix_unit(uint64_t i);

int oracle_num_threads(void);
/* Threads of the oracle's parallel loops from now on (n >= 1; results do not
 * depend on it: reductions run in fixed chunks summed in chunk order). */
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
