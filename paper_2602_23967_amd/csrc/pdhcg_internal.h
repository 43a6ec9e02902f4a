// pdhcg_internal.h -- device-side data layout shared by the host driver
// (host.cpp) and the gfx950 kernels (kernels.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "schedule.h"

namespace pdhcg {

struct CsrDev {
    int rows = 0, cols = 0;
    long long nnz = 0;
    int nparts = 1;            // > 1: column-partitioned (part-major storage)
    double* ypart = nullptr;   // nparts x rows partial row sums (partitioned only)
    int* rowptr = nullptr;     // nparts x (rows + 1), absolute offsets
    int* col = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;    // FP32 copy of val (mixed precision), same layout
    BlkDesc* blk = nullptr;
    int nblk = 0;
    double* seg_part = nullptr;
    int* lr_info = nullptr;    // per long row: {row, first segment slot, segment count}
    int nlr = 0;
    int nlr_coop = 0;          // the first nlr_coop long rows are summed by the whole block
    int lr0[3] = {-1, 0, 0};   // lr_info of the first long row (kernels read it without a load)
};

// inner-solver direction kinds
enum { DIR_PHI = 0, DIR_CONJ = 1, DIR_BETA = 2 };
// last inner step kinds
enum { STEP_NONE = 0, STEP_CG = 1, STEP_EXPAND = 2, STEP_PROP = 3 };

// Device control block: every scalar of the method lives here, so the
// whole iteration runs without host round trips.
struct Ctrl {
    // step sizes (Section 3.2)
    double omega, omega0, eta, tau, sigma, inv_tau;
    double norm_A, norm_Q;
    // inner tolerance (Section 3.3)
    double eps;
    double gamma_inner, eps_min, eps_fixed;
    // MPRGP state
    double abar, abar_scale, mprgp_gamma;
    double alpha, gam, pHp;
    double g_inv_tau;              // 1/tau of the subproblem the gradient g belongs to
    double gp2, b2, ptp;           // ||g^P||^2, ||beta||^2, phit'phi at the current x
    double res;                    // ||g^P|| at the last decision
    long long inner_it, inner_total, max_inner;
    // status sequence of the inner solve: the subproblem's base number (from
    // the host) and the inner steps that ran; step i posts seq_base + i, so
    // the inner-step kernels take no per-step argument (graph-capturable)
    long long seq_base, step;
    long long hp_active;           // launches of the inner product that did the product
    int done, need_g, skip_update, dir_mode, last_step, step_kind, proportional, pad0;
    // outer state (Sections 3.1-3.2)
    long long k, t, restarts, checks, max_iter;
    double theta;
    int use_halpern, store_delta, restart_pending, pad1;
    double ndx2, ndy2;             // ||x_T - x^k||^2, ||y_T - y^k||^2 of the last iteration
    double R_start, R_prev;
    int R_prev_valid, status, has_unbounded_x, pad2;
    double kp, ki, kd, pid_int, pid_prev;
    double rs_suff, rs_nec, rs_art;
    double tol, eps_inf;
    // check results (Section 4, 5)
    double pviol, py_sum, mvy2;            // A x_T side
    double dviol, qx_max, aty_max, c_max, xqx, cx, pr_sum, natural, mvx2;
    double r_primal, r_dual, r_gap, pobj, dobj;
    double bscale_p;                        // 1 + max(||lc||, ||uc||) over finite entries
    double ytil_max, ptil_sum, ptil_abs;    // primal-infeasibility pieces
    double w_viol, pw_sum, pw_abs;
    double d_max, cd, ad_viol, qd_max, gamma_q;
    int pinf, dinf, pad3, pad4;
    // power iteration
    double pw_norm;
};

// One side (lower or upper) of the variables' box.  Most problems share a
// few (l, u) pairs among all variables, so the bounds are kept as one
// constant (mode 1), a byte class per variable into a table of at most 256
// values (mode 2), or an array (mode 0): the inner steps then read one byte
// or nothing per variable instead of 16 bytes.  Exact: the same values.
struct BoundVec {
    const double* a = nullptr;            // mode 0: per variable
    const unsigned char* cls = nullptr;   // mode 2: class of each variable
    const double* tab = nullptr;          // mode 2: value of each class
    double k = 0.0;                       // mode 1: the value
    int mode = 0;
    __device__ __forceinline__ double operator[](long long i) const
    {
        return mode == 1 ? k : (mode == 2 ? tab[cls[i]] : a[i]);
    }
    // the same value with the storage mode known at compile time (the
    // inner step's kernels are compiled per mode: no branch per entry)
    template <int M>
    __device__ __forceinline__ double at(long long i) const
    {
        if constexpr (M == 1) return k;
        else if constexpr (M == 2) return tab[cls[i]];
        else return a[i];
    }
};

struct DevState {
    int n = 0, m = 0;
    CsrDev Q, A, AT;
    // Q = P + R'R given by its factors: Q holds [P | R'] (n x (n + k)), R is
    // k x n, and x_T, p, dx, v1, v2 carry k extra entries for R times them
    CsrDev R;
    int k = 0;
    int qdiag = 0;                 // Q diagonal (closed-form primal step)
    double* qd = nullptr;          // diagonal of Q (n)
    double *c = nullptr, *lc = nullptr, *uc = nullptr;
    BoundVec lv, uv;               // variable bounds (n)
    // iterates
    double *x = nullptr, *y = nullptr, *xa = nullptr, *ya = nullptr, *xt = nullptr, *yt = nullptr;
    // work vectors
    double *rhs = nullptr, *g = nullptr, *p = nullptr, *hp = nullptr, *aty = nullptr;
    double *dx = nullptr, *ytil = nullptr, *v1 = nullptr, *v2 = nullptr, *xbar = nullptr;
    // mixed precision: the reference point of the last check (x_ref, y_ref),
    // its FP64 products A x_ref, A' y_ref, and the FP32 differences
    // x_bar - x_ref, y - y_ref that the iteration's products gather
    int mixed = 0;
    double *xref = nullptr, *yref = nullptr, *axref = nullptr, *atyref = nullptr;
    float *dxb32 = nullptr, *dy32 = nullptr;
    Ctrl* ctrl = nullptr;
    double* partials = nullptr;
    double* partials2 = nullptr;   // partials of an epilogue whose finish is deferred
    // closed-form path, A with long rows: y of A's long rows after the last
    // dual step, two slots by iteration parity (2 x A.nlr)
    double* ylr = nullptr;
    hipEvent_t* tev = nullptr;             // when set: events around the next main kernel
    unsigned long long* dstat = nullptr;   // pinned status word (device view)
    // pinned check result (device view): (checks << 2) | restart << 1 | stop
    unsigned long long* dcheck = nullptr;
};

// ---- launchers (kernels.hip) ------------------------------------------------
// Every launcher enqueues on `s` and returns hipGetLastError().
hipError_t launch_init_start(const DevState& S, hipStream_t s);
// closed-form primal step fused with x_bar and the Halpern average of x
// the closed-form primal step; its finishing work is left for the dual
// step's finishing kernel when prox_diag_deferrable(S)
// tk: the round's step count t from the host (>= 0) or -1 (read ctrl->t);
// reduce = false: nothing reads this iteration's reductions (no partials,
// and the dual step's finishing kernel only completes long rows);
// lr_k >= 0: the dual step of iteration lr_k (round step lr_t) left its long
// rows, which this kernel's blocks complete first
hipError_t launch_prox_diag(const DevState& S, int store_delta, long long tk, bool reduce, long long lr_k,
                            long long lr_t, hipStream_t s);
bool prox_diag_deferrable(const DevState& S);
hipError_t launch_rhs(const DevState& S, hipStream_t s);
hipError_t launch_ginit(const DevState& S, long long seq, hipStream_t s);
// tail = R v for a factored Q (no-op otherwise); bulk: FP32 in mixed precision
hipError_t launch_tail(const DevState& S, const double* v, double* tail, bool bulk, hipStream_t s);
// rhs and warm-start gradient of the next subproblem from the previous one's
// gradient (no product with Q); starts the inner solve like launch_ginit
// pre_xbar: the previous iteration's x_bar kernel left its finishing work
// (the dual step ran without one)
hipError_t launch_rhs_grad(const DevState& S, long long seq, bool pre_xbar, hipStream_t s);
hipError_t launch_dir(const DevState& S, hipStream_t s);
hipError_t launch_hp(const DevState& S, hipStream_t s);
hipError_t launch_update(const DevState& S, hipStream_t s);
// x_bar = 2 x_T - x fused with the Halpern average of x
// x_bar and Halpern on x; its finishing work is always left for the dual
// step's finishing kernel (launch_dual with PRE_XBAR)
hipError_t launch_xbar(const DevState& S, int store_delta, long long tk, hipStream_t s);
hipError_t launch_clip(const DevState& S, double* x, hipStream_t s); // x <- proj_X(x)
// dual step and Halpern on y; pre names the earlier epilogue whose finishing
// work its finishing kernel runs first (same store_delta)
enum { PRE_NONE = 0, PRE_PROX = 1, PRE_XBAR = 2 };
// tk, kk: t and the iteration count k from the host (>= 0) or -1 (ctrl);
// leave_long: the closed-form path's non-reducing step leaves its long rows
// to the next launch_prox_diag (lr_k = kk, lr_t = tk) instead of a one-block
// finishing kernel (needs !reduce, no store_delta, PRE_PROX and S.ylr)
hipError_t launch_dual(const DevState& S, int store_delta, int pre, long long tk, long long kk, bool reduce,
                       bool leave_long, hipStream_t s);
// KKT pieces at (x, y); with `full` also the infeasibility certificates
// (and, with `dinf`, the unboundedness ones) and the solver's decision
hipError_t launch_check(const DevState& S, const double* x, const double* y, int full, int dinf,
                        hipStream_t s);
hipError_t launch_restart_copy(const DevState& S, hipStream_t s);
// mixed precision only (no-ops otherwise): take (x_T, y_T) as the new
// reference point after a check; zero the reference before the first check
hipError_t launch_ref_update(const DevState& S, hipStream_t s);
hipError_t launch_ref_zero(const DevState& S, hipStream_t s);
// power iteration pieces: v <- unit start vector; w = M v with ||w||^2; v = w / ||w||
hipError_t launch_power_start(const DevState& S, double* v, int len, hipStream_t s);
hipError_t launch_spmv_norm(const DevState& S, const CsrDev& M, const double* x, double* y,
                            hipStream_t s);
hipError_t launch_scale(const DevState& S, double* v, int len, hipStream_t s);
// operator-level entry points
hipError_t launch_spmv_plain(const DevState& S, const CsrDev& M, const double* x, double* y,
                             hipStream_t s);
hipError_t launch_dot(const DevState& S, const double* a, const double* b, int len,
                      hipStream_t s);

int vec_grid(long long len);

// ---- batched solve of many QPs with diagonal Q (batch.hip) ----------------------

// launch shape of the batched kernels: threads per workgroup (one instance
// per workgroup) and doubles of LDS for an instance's staged operands
struct BatchShape {
    int threads, lds, waves_per_simd;
};
// the table of compiled shapes (*count entries)
const BatchShape* batch_shapes(int* count);
constexpr int BATCH_SHAPE_DEFAULT = 12;          // 256 threads, 4992 doubles, 4 waves per SIMD
// the per-instance norm kernel's shape (its values do not depend on the LDS
// size, and 3 workgroups per CU measured faster than 4: 99 against 153 ms
// for the 4096-instance MPC batch)
constexpr int BATCH_SHAPE_NORM = 1;
constexpr int BATCH_SHAPE_GENERAL_DEFAULT = 8;   // 1024 threads, 12288 doubles (inner solves)

struct BatchOut {
    int status, pad;
    long long iterations, restarts, inner_iterations;
    double r_primal, r_dual, r_gap, pobj, dobj, omega, ytil_max, d_max;
    // device wall clock (wall_clock64 ticks) when a workgroup took the
    // instance and when it finished it
    unsigned long long t_start, t_end;
};

struct BatchParams {
    double tol, eps_inf, theta, kp, ki, kd, rs_suff, rs_nec, rs_art;
    double gamma_inner, eps_min, eps_fixed, mprgp_gamma, abar_scale;
    long long max_iter, check_every, max_inner;
    int use_halpern, pad;
};

struct BatchDev {
    int count = 0;
    int* queue = nullptr;                       // work counter (instances taken)
    const int* order = nullptr;                 // queue position -> instance (NULL: index order)
    const int *voff = nullptr, *roff = nullptr; // count + 1 each
    const int *arp = nullptr, *acol = nullptr;  // A, global indices
    const double* aval = nullptr;
    const int *trp = nullptr, *tcol = nullptr;  // A'
    const double* tval = nullptr;
    const int *qrp = nullptr, *qcol = nullptr;  // Q (block-diagonal, global indices)
    const double* qval = nullptr;
    // the columns of A, A' and Q as 16-bit indices local to the instance
    // (all three set when every instance has n_b, m_b < 65536, else NULL)
    const unsigned short *acol16 = nullptr, *tcol16 = nullptr, *qcol16 = nullptr;
    // FP32 copies of the values for the bulk products of a mixed-precision
    // solve (all NULL in FP64)
    const float *aval32 = nullptr, *tval32 = nullptr, *qval32 = nullptr;
    const double *qd = nullptr, *c = nullptr, *lc = nullptr, *uc = nullptr;
    BoundVec lv, uv;                            // variable bounds (n), as for one problem
    // per instance
    const double *eta = nullptr, *omega0 = nullptr, *cmax = nullptr, *bscale = nullptr, *gammaq = nullptr;
    const double* normq = nullptr;              // ||Q_b||_2 (x 1.01 for a non-diagonal Q_b)
    const int* unb = nullptr;
    const int* qgen = nullptr;                  // 1: Q_b not diagonal (inner CG solve)
    // state (packed like the problem)
    double *x = nullptr, *y = nullptr, *xa = nullptr, *ya = nullptr, *xt = nullptr, *yt = nullptr;
    double *xbar = nullptr, *aty = nullptr, *d = nullptr, *ytil = nullptr;
    double *rhs = nullptr, *g = nullptr, *p = nullptr, *hp = nullptr;
    // mixed precision: the reference point of the last check and A x_ref
    double *xref = nullptr, *yref = nullptr, *axref = nullptr;
    BatchOut* out = nullptr;
};

// persistent grid of a shape (which: 0 FP64 solve, 1 mixed solve, 2 norm):
// the workgroups the device holds at once, at most `count`
int batch_grid(int shape, int which, int count);
// ||M_b||_2 per instance by power iteration on M_b'M_b: M (rows given by
// rowoff, columns by coloff) and its transpose Mt; instances with sel[b] == 0
// get 0 (sel may be NULL)
hipError_t launch_batch_norm(const BatchDev& B, int shape, const int* rowoff, const int* coloff,
                             const int* mrp, const int* mcol, const double* mval,
                             const int* trp, const int* tcol, const double* tval, const int* sel,
                             double tol, long long max_iter, double* v, double* w, double* u,
                             double* out, hipStream_t s);
hipError_t launch_batch_solve(const BatchDev& B, const BatchParams& P, int shape, hipStream_t s);
// dst[i] = (float)src[i]
hipError_t launch_to_f32(const double* src, float* dst, long long len, hipStream_t s);

}  // namespace pdhcg
