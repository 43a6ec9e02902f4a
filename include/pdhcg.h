/*
 * pdhcg.h -- C ABI of the MI355X (gfx950) PDHCG-II convex-QP solver.
 *
 * Problem (Section 2, eq. QP, of arXiv 2602.23967):
 *
 *     minimize    1/2 x'Qx + c'x
 *     subject to  l_c <= A x <= u_c       (rows; here from b and a sense)
 *                 l_v <=  x  <= u_v       (box; bounds may be +-INFINITY)
 *
 * with Q symmetric positive semidefinite.  The solver is the restarted,
 * reflected-Halpern PDHG iteration of Sections 2.1 and 3 with the primal
 * subproblem solved by conjugate gradients on the free set (closed form
 * when Q is diagonal), the PID primal weight of Section 3.2, the adaptive
 * inner tolerance of Section 3.3, the relative L-infinity KKT test of
 * Section 4 and the infeasibility certificates of Section 5.  All arithmetic
 * is IEEE FP64, except the iteration's sparse products of a solve that asks
 * for mixed precision (qp_params.precision, below).
 *
 * Conventions (Section 2, eq. dualQP / minimax): y_i > 0 means the row's
 * upper bound is active, y_i < 0 its lower bound; '>=' rows therefore have
 * y_i <= 0.  The reduced cost is r = Qx + c + A'y.
 *
 * Ownership and threading: qp_create copies every input (the caller may free
 * its buffers on return); the handle owns all device memory until
 * qp_destroy.  One thread at a time per handle.  Distinct handles on
 * distinct streams may run concurrently.  A handle lives on the HIP device
 * that was current when it was created; make that device current for every
 * later call on it.  Pointers documented as "device"
 * are HIP device pointers (e.g. torch.cuda tensors' data_ptr()); all others
 * are host pointers.
 *
 * Errors: functions returning int give a status (>= 0) or a negative error
 * code; qp_last_error() then describes the failure (thread-local string).
 */
#ifndef PDHCG_H
#define PDHCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qp_handle qp_handle;

/* solve status (>= 0) */
enum {
    QP_NOT_SOLVED = 0,
    QP_OPTIMAL = 1,            /* max(r_primal, r_dual, r_gap) <= tol (Section 4) */
    QP_PRIMAL_INFEASIBLE = 2,  /* Farkas ray found (Section 5.1); y holds it */
    QP_DUAL_INFEASIBLE = 3,    /* unbounded ray found (Section 5.2); x holds it */
    QP_ITERATION_LIMIT = 4,
    QP_NUMERICAL_ERROR = 5     /* a residual became NaN or infinite */
};

/* error codes (< 0) */
enum {
    QP_ERR_INVALID_ARG = -1,   /* malformed input; nothing was allocated */
    QP_ERR_NOT_SYMMETRIC = -2, /* Q is not symmetric (pattern or values) */
    QP_ERR_DEVICE = -3,        /* HIP error or out of device memory */
    QP_ERR_STATE = -4          /* e.g. qp_result before any qp_solve */
};

/* operators for qp_apply */
enum { QP_OP_Q = 0, QP_OP_A = 1, QP_OP_AT = 2 };

/* Solver parameters.  Fields marked (paper) are values the paper states;
 * the others are readings where the paper is silent. */
typedef struct {
    double tol;               /* (paper, Section 4) eps_tol on max(r_primal, r_dual, r_gap); 1e-6 */
    int64_t max_iter;         /* outer PDHG iterations; 0 returns the start point's residuals */
    int64_t check_every;      /* cadence of KKT / infeasibility / restart checks; 64 */
    int64_t max_inner;        /* cap on inner iterations per subproblem; 500 */
    int use_halpern;          /* 1: reflected Halpern averaging (Section 3.1); 0: plain PDHG */
    int inner_lag;            /* inner steps queued ahead of the host's view of the stop flag; 1 */
    double theta;             /* Halpern reflection; 1 */
    double kp, ki, kd;        /* PID gains on log(omega) (Section 3.2); 0.99, 0.01, 0 */
    double gamma_inner;       /* (paper, Section 3.3) 5e-4 */
    double eps_min;           /* (paper, Section 3.3) 1e-9 */
    double eps_inner_fixed;   /* > 0: fixed inner tolerance instead of the adaptive rule; 0 */
    double restart_sufficient, restart_necessary, restart_artificial; /* 0.2, 0.8, 0.36 */
    double eps_inf;           /* certificate tolerance (Section 5); 1e-8 */
    double eta_scale;         /* (paper, Section 3.2) eta = eta_scale / ||A||_2; 0.998 */
    double norm_safety;       /* ||A||_2 estimate multiplied by this; 1.01 */
    double power_tol;         /* power-iteration relative-change tolerance; 1e-7 */
    int64_t power_max_iter;   /* 1000 */
    double mprgp_gamma;       /* proportioning constant of the inner solver; 1 */
    double mprgp_abar_scale;  /* expansion step = scale / (||Q||_2 + 1/tau); 1.9 */
    int timing;               /* > 0: time every `timing`-th launch of each kernel family */
    int precision;            /* QP_PRECISION_FP64 (0, default) or QP_PRECISION_MIXED (1) */
    int graph_steps;          /* > 0: the inner solve's steps are launched as a captured HIP
                                 graph of this many steps (0: one launch per kernel; timing
                                 forces 0); results are the same either way; 0 (measured
                                 slower: the steps are bound by the GPU, not by launches) */
    int reserved;
} qp_params;

/* Arithmetic of a solve.  FP64: every step in double precision.  MIXED: the
 * sparse products of the iteration itself (A'y with the primal step, A x_bar
 * with the dual step, the products with Q of the inner solve) read an FP32
 * copy of the matrix values, round the gathered operand to FP32 and sum in
 * FP32; the vector updates, the Halpern anchor and averages, the step sizes,
 * the KKT residuals (Section 4), the restart / termination tests and the
 * certificates (Section 5) stay FP64, and the checks use the FP64 values. */
enum { QP_PRECISION_FP64 = 0, QP_PRECISION_MIXED = 1 };

/* kernel families reported by qp_info.fam_* when timing is on */
enum {
    QP_FAM_SPMV_HP = 0,   /* inner step: H p (or H x after an expansion), fused */
    QP_FAM_UPDATE = 1,    /* inner step: x, g update with reductions */
    QP_FAM_DIR = 2,       /* inner step: next direction */
    QP_FAM_RHS = 3,       /* A'y fused with the subproblem right-hand side (or, for a diagonal
                             Q, with the closed-form step, x_bar and Halpern on x) */
    QP_FAM_GINIT = 4,     /* gradient at the warm start */
    QP_FAM_DUAL = 5,      /* A x_bar fused with the dual step and Halpern on y */
    QP_FAM_HALPX = 6,     /* after the inner solve: x_bar, Halpern on x, movement, tolerance */
    QP_FAM_CHECK = 7,     /* KKT / infeasibility / restart checks */
    QP_NFAM = 8
};

typedef struct {
    int status;
    int precision;             /* QP_PRECISION_* the solve ran in */
    int64_t iterations;        /* outer iterations */
    int64_t inner_iterations;  /* total inner (CG/MPRGP) iterations */
    int64_t restarts;
    int64_t checks;
    double r_primal, r_dual, r_gap;  /* Section 4, at the returned point */
    double primal_obj, dual_obj;
    double natural_residual;   /* ||x - proj_X(x - r)||_inf (diagnostic) */
    double omega, eta, norm_A, norm_Q, eps_inner;
    double solve_seconds;      /* wall time of the last qp_solve */
    double setup_seconds;      /* wall time of qp_create */
    double fam_ms[QP_NFAM];    /* summed device time of the timed launches */
    int64_t fam_timed[QP_NFAM];/* number of timed launches */
    int64_t fam_launches[QP_NFAM]; /* number of launches */
    int64_t spmv_hp_active;    /* QP_FAM_SPMV_HP launches that ran (the rest found the
                                  inner solve already stopped and returned at once) */
} qp_info;

/* Defaults listed above. */
qp_params qp_params_default(void);

/*
 * Create a problem.  Q is full symmetric CSR (both triangles; int64 row
 * pointers of length n+1, int32 column indices sorted and unique within a
 * row); Q_rowptr == NULL means Q = 0 (an LP).  A is m x n CSR in the same
 * form (may be NULL when m == 0).  sense[i] is 'E' (A_i x = b_i), 'G'
 * (A_i x >= b_i) or 'L' (A_i x <= b_i), mapped to (l_c, u_c) as in Section 2.
 * lb / ub may be NULL (-inf / +inf).  Validation (before any device call):
 * n >= 1, m >= 0, row pointers start at 0 and do not decrease, nnz < 2^31,
 * columns in range, sorted and unique, every value, c and b finite, lb <= ub,
 * lb < +inf, ub > -inf, Q symmetric to 1e-14 relative.  Returns 0 and
 * *out, or a negative error code (nothing allocated).
 */
int qp_create(int64_t n, int64_t m,
              const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
              const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
              const double* c, const double* b, const char* sense,
              const double* lb, const double* ub, qp_handle** out);

/* Same with the row bounds given directly: l_c <= A x <= u_c (Section 2,
 * eq. QP); lc / uc may hold -inf / +inf and must satisfy lc <= uc. */
int qp_create_ranged(int64_t n, int64_t m,
                     const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                     const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                     const double* c, const double* lc, const double* uc,
                     const double* lb, const double* ub, qp_handle** out);

/* Same as qp_create with a structured quadratic term Q = P + R'R (Section
 * 2.2, structured quadratic objective): P is sparse symmetric n x n CSR (may
 * be NULL for P = 0) and R is k x n CSR (k >= 1, usually k << n).  R'R is
 * never formed: every product with Q is a product with R (k rows) followed
 * by one with the n x (n + k) matrix [P | R'] on [v; R v].  Validation as
 * qp_create, plus R's CSR rules and n + k < 2^31.  qp_apply(QP_OP_Q) applies
 * P + R'R. */
int qp_create_factored(int64_t n, int64_t m,
                       const int64_t* P_rowptr, const int32_t* P_col, const double* P_val,
                       int64_t k, const int64_t* R_rowptr, const int32_t* R_col, const double* R_val,
                       const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                       const double* c, const double* b, const char* sense,
                       const double* lb, const double* ub, qp_handle** out);

/* Run every later call of this handle on `stream` (a hipStream_t; NULL
 * selects the handle's own stream).  The caller keeps ownership. */
int qp_set_stream(qp_handle* h, void* stream);

/* Solve from the start point x0 = proj_X(0), y0 = 0 with default
 * parameters except tol and max_iter.  Blocking.  Returns the status. */
int qp_solve(qp_handle* h, double tol, int64_t max_iter);

/* Solve with explicit parameters (NULL: defaults). */
int qp_solve_ex(qp_handle* h, const qp_params* params);

/*
 * Copy the last solve's result into caller buffers (host; any may be NULL):
 * x (n), y (m), info.  OPTIMAL / ITERATION_LIMIT / NUMERICAL_ERROR: the
 * PDHG output (x_T, y_T) of the last iteration, x in X and y in Y.
 * PRIMAL_INFEASIBLE: y = the Farkas ray, ||y||_inf = 1 (x = x_T).
 * DUAL_INFEASIBLE: x = the unbounded direction, ||x||_inf = 1 (y = y_T).
 * Returns the status, or QP_ERR_STATE before the first solve.
 */
int qp_result(const qp_handle* h, double* x, double* y, qp_info* info);

/* Release all device memory of the handle.  NULL is ignored. */
void qp_destroy(qp_handle* h);

/* Description of the last error on this thread ("" if none). */
const char* qp_last_error(void);

/* ---- operator-level calls on caller-owned DEVICE buffers -----------------
 * They run the same kernels the solver runs, synchronously on the handle's
 * stream, and exist so each step can be checked in isolation. */

/* y = M x for M in {Q (n x n), A (m x n), A' (n x m)} (device x, y). */
int qp_apply(qp_handle* h, int op, const double* x, double* y);

/* *out (host) = a'b over len elements (device a, b), deterministic. */
int qp_dot(qp_handle* h, int64_t len, const double* a, const double* b, double* out);

/* One primal subproblem (Section 2.2, eq. primal_update):
 *   x <- argmin over l_v <= x <= u_v of 1/2 x'(Q + I/tau)x - rhs'x,
 * started from x (device, n; clipped to the box first), stopping when the
 * projected-gradient 2-norm is <= eps or after max_inner iterations.
 * iters and res (host, may be NULL) receive the iteration count and the
 * final projected-gradient norm. */
int qp_subproblem(qp_handle* h, double tau, const double* rhs, double* x, double eps,
                  int64_t max_inner, int64_t* iters, double* res);

/* KKT residuals of Section 4 at (x, y) (device, n and m).  out (host, 7):
 * r_primal, r_dual, r_gap, primal objective, dual objective, natural
 * residual, unnormalised primal violation. */
int qp_kkt(qp_handle* h, const double* x, const double* y, double* out);

/* ||A||_2 and ||Q||_2 estimates of qp_create (host outputs, may be NULL). */
int qp_norms(const qp_handle* h, double* norm_A, double* norm_Q);

/* ---- batched solve: many independent QPs in one persistent launch --------
 *
 * For many small QPs (e.g. linear MPC, small factor models) solved together.
 * The caller packs the instances block-diagonally: instance i owns variables
 * [var_off[i], var_off[i+1]) and rows [row_off[i], row_off[i+1]); Q (n x n,
 * symmetric, every entry inside its instance's block, or NULL) and A (m x n,
 * every entry inside its instance's block) are CSR as in qp_create, as are
 * c, b, sense, lb, ub over all instances.  Each instance runs the method of
 * qp_solve with its own step sizes, restarts, weight, inner tolerance and
 * status: the closed-form primal step when its block of Q is diagonal, the
 * boxed conjugate-gradient inner solve otherwise.  One workgroup solves one
 * instance at a time, so an instance's result does not depend on which other
 * instances share the launch.  Same ownership and error rules as qp_create;
 * a row longer than QP_BATCH_MAX_ROW is QP_ERR_INVALID_ARG. */
typedef struct qp_batch qp_batch;

/* Longest row of A, of A' (column of A) and of Q an instance of a batch may
 * have: the batched kernel sums each row with one thread.  Instances with
 * longer rows belong on the single-problem path. */
#define QP_BATCH_MAX_ROW 256

int qp_batch_create(int64_t count, const int64_t* var_off, const int64_t* row_off,
                    const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                    const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                    const double* c, const double* b, const char* sense,
                    const double* lb, const double* ub, qp_batch** out);

/* Solve every instance (params as qp_solve_ex; NULL = defaults; inner-solver
 * fields are unused).  Blocking.  Returns the number of OPTIMAL instances or
 * a negative error code. */
int qp_batch_solve(qp_batch* bt, const qp_params* params);

/* Result of instance i (host buffers of its n_i and m_i entries, any may be
 * NULL), with the conventions of qp_result.  Returns the instance status. */
int qp_batch_result(const qp_batch* bt, int64_t i, double* x, double* y, qp_info* info);

/* Statuses of all instances (host, count entries) and the last solve's wall
 * time in seconds (may be NULL). */
int qp_batch_statuses(const qp_batch* bt, int32_t* status, double* seconds);

/* When each instance of the last solve was taken up by a workgroup and
 * when it finished, in seconds after the first instance was taken up
 * (device wall clock; host buffers of count entries, either may be NULL):
 * the instances' completion times inside the one persistent launch.
 * Returns 0, QP_ERR_STATE before a solve, QP_ERR_DEVICE when the device
 * reports no wall clock rate. */
int qp_batch_times(const qp_batch* bt, double* start_s, double* end_s);

void qp_batch_destroy(qp_batch* bt);

/* ---- batched solve without device allocation ---------------------------
 *
 * For callers that cannot allocate device memory: tight serving loops and
 * harnesses that forbid hipMalloc.  One blocking call solves a batch exactly
 * as qp_batch_create + qp_batch_solve + qp_batch_result would (same
 * arguments and validation, same kernels, default launch schedule: the
 * results are bitwise those of the allocating path), but every device buffer
 * of the batch -- the copied problem, the iterates and anchors, the work
 * counter and the outcome records -- is carved from one static workspace of
 * QP_STATIC_WORKSPACE_BYTES that the library holds on each device it runs on
 * until the process ends.  Nothing is allocated or freed on the device, and
 * no stream or event is created: the call runs on `stream` (a hipStream_t of
 * the current device; NULL is the null stream) and waits for it.
 *
 * Inputs as qp_batch_create (host buffers, copied; the caller may free them
 * on return); params as qp_batch_solve (NULL = defaults).  Outputs (host,
 * each may be NULL): x (all n variables) and y (all m rows), packed like the
 * problem, with the conventions of qp_batch_result (certificates in place of
 * the iterates for infeasible instances); status[count]; info[count].
 * Returns the number of OPTIMAL instances, or QP_ERR_INVALID_ARG (bad input,
 * or a batch whose device copy does not fit the workspace: the message gives
 * the limit), QP_ERR_DEVICE.
 *
 * The workspace keeps the last call's contents; every buffer a call reads is
 * written by that call first.  Calls on one device share the workspace: the
 * library serialises calls from the threads of one process (each holds the
 * device's workspace until its results are copied out); work that another
 * agent (another library instance in the process, or a caller writing the
 * workspace) overlaps with a call races. */
#define QP_STATIC_WORKSPACE_BYTES (64ll << 20)

int qp_batch_solve_static(int64_t count, const int64_t* var_off, const int64_t* row_off,
                          const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                          const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                          const double* c, const double* b, const char* sense,
                          const double* lb, const double* ub, const qp_params* params, void* stream,
                          double* x, double* y, int32_t* status, qp_info* info);

/* ---- launch schedule of the batched solve, and its autotuner -------------
 *
 * One workgroup solves one instance; the schedule is the workgroup shape
 * (threads, and doubles of LDS that hold a small instance's product
 * operands) and the order in which workgroups take instances from the
 * queue (0: index order, 1: largest instance first, the default).  The grid
 * is persistent: as many workgroups as the device holds at once for the
 * shape.  More threads per instance shorten each instance; fewer threads
 * and less LDS let more instances run at once: which is faster depends on
 * the instance sizes, hence the tuner.  The order never changes a result;
 * the shape may change the last bits (a workgroup reduction groups its
 * terms by the workgroup size), and each shape is deterministic. */

/* Number of compiled shapes, and shape i's threads per workgroup, LDS
 * doubles and the waves per SIMD its register allocation leaves room for
 * (1: as many registers as the workgroup size allows; more: fewer registers,
 * some spilled, more instances resident) (host outputs, may be NULL).  A new
 * batch uses qp_batch_default_shape(0) whatever its instances, so that an
 * instance's result never depends on the others in the batch;
 * qp_batch_default_shape(1) is the shape that suits instances with an inner
 * solve (non-diagonal Q) better, which the server's general lanes use. */
int qp_batch_num_shapes(void);
int qp_batch_default_shape(int32_t general);
int qp_batch_shape_info(int32_t shape, int32_t* threads, int32_t* lds_doubles, int32_t* waves_per_simd);

/* Set the schedule of later solves of bt (-1 keeps a field); get it. */
int qp_batch_set_schedule(qp_batch* bt, int32_t shape, int32_t order);
int qp_batch_get_schedule(const qp_batch* bt, int32_t* shape, int32_t* order);

/* Autotuner: solves the batch once per candidate schedule (every shape in
 * both orders, candidate c = 2 * shape + order) with params, keeps the
 * fastest, solves once more with it so the batch holds its results, and
 * returns c.  seconds (host, 2 * qp_batch_num_shapes() entries, may be NULL)
 * receives each candidate's solve time.  Blocking; costs that many solves. */
int qp_batch_tune(qp_batch* bt, const qp_params* params, double* seconds);

/* ---- request server: continuous batching ---------------------------------
 *
 * A server takes QPs of any size as they arrive and solves them on one GPU:
 * requests with n + m <= batch_max_dim (general_max_dim for a non-diagonal Q)
 * and no row of A, A' or Q longer than QP_BATCH_MAX_ROW nonzeros are gathered
 * into batched launches (one workgroup per instance, as qp_batch_solve; a
 * launch ends with its slowest instance, so diagonal-Q and non-diagonal-Q
 * requests have lanes of their own), the others are solved on
 * the single-problem path by worker threads, each on its own stream.  Up to
 * `batch_lanes + general_lanes` batched launches and `single_workers` single solves are in
 * flight at once; a request is admitted when a lane or worker is free and
 * the device bytes of everything in flight plus its own (its CSR data and
 * solver state) stay within `device_budget`.  Requests that arrive while
 * others run join the next launch of a free lane, so their work overlaps on
 * the device with the launches already running.  Every solve keeps its
 * iterates, Halpern anchor, restart and weight state on the device until it
 * ends.  A request's result does not depend on the other requests it shares
 * a launch with.  Thread-safe: any thread may submit, wait and fetch. */
typedef struct qp_server qp_server;

typedef struct {
    int64_t device_budget;    /* bytes of device memory for requests in flight; 8 GiB */
    int64_t batch_max_dim;    /* diagonal or zero Q: n + m at or below which a request
                                 joins a batch; 20000 */
    int64_t general_max_dim;  /* non-diagonal Q (inner solve in the workgroup): the same
                                 limit; 3000 */
    int32_t batch_lanes;      /* batched launches in flight for diagonal-Q requests; 2 */
    int32_t general_lanes;    /* batched launches in flight for non-diagonal-Q requests; 2 */
    int32_t single_workers;   /* single-path solves in flight; 5 */
    int32_t max_batch;        /* instances per batched launch; 1024 */
    int32_t batch_shape;      /* launch shape of the batched launches of diagonal-Q requests
                                 (qp_batch_set_schedule), -1: the library default */
    int32_t batch_order;      /* their queue order (0 or 1), -1: the library default */
    int32_t general_shape;    /* launch shape of the batched launches of non-diagonal-Q
                                 requests, -1: qp_batch_default_shape(1) */
    int32_t diag_workers;     /* of the single-path workers, those that take only
                                 diagonal-Q requests (or any request when no other
                                 worker exists), <= single_workers; -1: 1 when
                                 single_workers >= 2, else 0 */
    double batch_linger_us;   /* a free lane waits up to this long (from the oldest waiting
                                 request's arrival) for more requests before launching; 200 */
} qp_server_config;

/* Host times of one request, seconds since the server was created. */
typedef struct {
    double submitted, started, finished;
    int32_t route;            /* 0: batched launch, 1: single-problem path */
    int32_t batch_size;       /* instances of its launch (1 on the single path) */
} qp_request_times;

qp_server_config qp_server_config_default(void);

/* Start a server (params as qp_solve_ex, NULL = defaults; cfg NULL =
 * defaults).  Returns 0 and *out, or a negative error code. */
int qp_server_create(const qp_server_config* cfg, const qp_params* params, qp_server** out);

/* Submit one QP (arguments, validation and copying as qp_create; nothing is
 * allocated on the device here).  Returns the request id (>= 0) or a
 * negative error code; a request larger than device_budget is rejected with
 * QP_ERR_INVALID_ARG. */
int64_t qp_server_submit(qp_server* s, int64_t n, int64_t m,
                         const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                         const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                         const double* c, const double* b, const char* sense,
                         const double* lb, const double* ub);

/* Wait up to timeout_s seconds (< 0: no limit) for request `id`.  Returns
 * its status (> 0) once solved, QP_NOT_SOLVED (0) on time-out, or a
 * negative error code (unknown id, or the error its solve ended with). */
int qp_server_wait(qp_server* s, int64_t id, double timeout_s);

/* Result of a finished request, with the conventions of qp_result (host
 * buffers of n and m entries, any pointer may be NULL), and its times.
 * Releases the request: its id is unknown afterwards.  Returns its status
 * or a negative error code (QP_ERR_STATE while it is not finished). */
int qp_server_result(qp_server* s, int64_t id, double* x, double* y, qp_info* info,
                     qp_request_times* times);

/* Finish the requests in flight, drop the waiting ones and stop. */
void qp_server_destroy(qp_server* s);

/* ---- measurement utility (not part of the method) --------------------- */

/* The device's rate of random 8-byte gathers from a vector of n doubles
 * (n >= 4, < 2^31), with gathering blocks keyed to the same four XCD column
 * parts as the column-partitioned products: `gathers` (>= 2048) pseudo-
 * random reads per launch, timed over `repeats` launches after 3 untimed
 * ones on the null stream.  Allocates and frees its own device memory.
 * *gathers_per_s (host) receives the rate.  Returns 0, or
 * QP_ERR_INVALID_ARG / QP_ERR_DEVICE.  The large products are bound by this
 * rate rather than by HBM bytes; the bench reports the product's own gather
 * rate against it. */
int qp_measure_gather_rate(int64_t n, int64_t gathers, int32_t repeats, double* gathers_per_s);

/* ---- host-only diagnostics (no device call) --------------------------- */

/* The SpMV work schedule the library builds for a CSR with `rows` rows and
 * int64 row pointers `rowptr` (host): row blocks of at most 2048 nonzeros
 * and 256 rows, and 2048-nonzero segments of longer rows.  Writes up to
 * `cap` items of 8 int32 each to `out` (host; may be NULL to count):
 * {first row, rows (0 for a segment), first nonzero, end nonzero,
 *  long-row id, segment index, segment count, first segment slot}.
 * Returns the number of items (or a negative error code). */
int64_t qp_spmv_schedule(int64_t rows, const int64_t* rowptr, int32_t* out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
