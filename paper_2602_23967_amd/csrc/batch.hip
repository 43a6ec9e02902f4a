// batch.hip -- many independent QPs with a diagonal (or zero) Q solved in one
// persistent launch.
//
// The instances are packed block-diagonally (variables and rows of instance b
// are the ranges [voff[b], voff[b+1]) and [roff[b], roff[b+1])).  Each
// workgroup takes the next instance from a work counter and runs the whole
// method on it: the closed-form primal step (Section 2.2, diagonal Hessian),
// the dual step (eqs. extrapolation, dual_update), the reflected Halpern
// average (Section 3.1), the KKT test (Section 4), the certificates
// (Section 5), the restart rule and the PID weight (Section 3.2) -- with its
// own step sizes, restart state and status.  All reductions are workgroup
// reductions broadcast to every thread, so every thread takes the same
// decisions; nothing waits on another workgroup, and the only device-scope
// atomic is the work counter, taken once per instance.
#include <math.h>

#include <atomic>

#include "device_math.h"
#include "pdhcg_internal.h"

namespace pdhcg {

// a value every lane holds identically, moved to scalar registers
__device__ __forceinline__ double uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum (bit j of MAXMASK clear) or max (bit set) of NR values over the
// workgroup, in a fixed order; the result lands in every thread.
template <int NR, unsigned MAXMASK, int NT>
__device__ void wg_reduce(double (&v)[NR], double* lds)
{
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int kind = ((MAXMASK >> j) & 1u) ? R_MAX : R_SUM;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[j] = rcomb(kind, v[j], __shfl_xor(v[j], off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NR; ++j) lds[wave * NR + j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int kind = ((MAXMASK >> j) & 1u) ? R_MAX : R_SUM;
        double r = lds[j];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = rcomb(kind, r, lds[w * NR + j]);
        v[j] = uniform(r);
    }
    __syncthreads();
}

// sums of slots 0 and 1, minimum of slot 2, over the workgroup (in every thread)
template <int NT>
__device__ void wg_reduce_min3(double (&v)[3], double* lds)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int kind = j == 2 ? R_MIN : R_SUM;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[j] = rcomb(kind, v[j], __shfl_xor(v[j], off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) lds[wave * 3 + j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int kind = j == 2 ? R_MIN : R_SUM;
        double r = lds[j];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = rcomb(kind, r, lds[w * 3 + j]);
        v[j] = uniform(r);
    }
    __syncthreads();
}

// one instance's side of the box: entry i of the instance starting at off
struct BoundAt {
    BoundVec b;
    int off;
    __device__ __forceinline__ double operator[](int i) const { return b[(long long)off + i]; }
};

// Column indices of a packed matrix: global 32-bit ones, or 16-bit indices
// local to the instance (column = off + local), which cut the index bytes
// of every product in half when every instance has fewer than 65536
// variables and rows.  at(q, off) is the global column of entry q.
template <bool C16>
struct Cols {
    const int* g;
    const unsigned short* l;
    __device__ __forceinline__ int at(int q, int off) const
    {
        if constexpr (C16) return off + (int)l[q];
        else return g[q];
    }
    // the column relative to off (an index into an LDS copy of the operand)
    __device__ __forceinline__ int rel(int q, int off) const
    {
        if constexpr (C16) return (int)l[q];
        else return g[q] - off;
    }
};

template <bool C16>
__device__ __forceinline__ double row_dot(const int* rp, Cols<C16> col, const double* val,
                                          const double* x, int row, int off)
{
    double s = 0.0;
    for (int q = rp[row]; q < rp[row + 1]; ++q) s += val[q] * x[col.at(q, off)];
    return s;
}

// A bulk product of the iteration.  FP64: the row of M times x.  Mixed
// precision: the product is split around a reference point x_ref whose
// product ref = (M x_ref)_row is known in FP64 (from the last check):
// ref + M (x - x_ref) with FP32 values, the difference rounded to FP32 and
// an FP32 sum, so the FP32 rounding scales with the movement since the
// check and not with the iterate.
template <bool F32, bool C16>
__device__ __forceinline__ double row_dot_bulk(const int* rp, Cols<C16> col, const double* val,
                                               const float* val32, const double* x, const double* xref,
                                               double ref, int row, int off)
{
    if constexpr (F32) {
        float s = 0.0f;
        for (int q = rp[row]; q < rp[row + 1]; ++q) {
            const int j = col.at(q, off);
            s += val32[q] * (float)(x[j] - xref[j]);
        }
        return ref + (double)s;
    } else {
        return row_dot(rp, col, val, x, row, off);
    }
}

template <int NT, int LDSN>
__device__ double power_norm_wg(int c0, int n, int r0, int m, const int* mrp, const int* mcol,
                                const double* mval, const int* trp, const int* tcol, const double* tval,
                                double tol, long long max_iter, double* v, double* w, double* u, double* lds,
                                double* sbuf);

// The same product with the operand staged in the workgroup's LDS (sv[j -
// off] holds the operand, or in mixed precision its difference from the
// reference point): identical arithmetic, LDS gathers instead of L2 ones.
template <bool F32, bool C16>
__device__ __forceinline__ double row_dot_lds(const int* rp, Cols<C16> col, const double* val,
                                              const float* val32, const double* sv, int off, double ref,
                                              int row)
{
    if constexpr (F32) {
        float s = 0.0f;
        for (int q = rp[row]; q < rp[row + 1]; ++q) s += val32[q] * (float)sv[col.rel(q, off)];
        return ref + (double)s;
    } else {
        double s = 0.0;
        for (int q = rp[row]; q < rp[row + 1]; ++q) s += val[q] * sv[col.rel(q, off)];
        return s;
    }
}

// the inner step's product H p: FP32 values, direction and sum in mixed
// precision (the inner solve re-forms its gradient in FP64 at every
// subproblem and after every expansion step)
template <bool F32, bool C16>
__device__ __forceinline__ double hp_dot(const int* rp, Cols<C16> col, const double* val,
                                         const float* val32, const double* x, int row, int off)
{
    if constexpr (F32) {
        float s = 0.0f;
        for (int q = rp[row]; q < rp[row + 1]; ++q) s += val32[q] * (float)x[col.at(q, off)];
        return (double)s;
    } else {
        return row_dot(rp, col, val, x, row, off);
    }
}

// ---- ||M_b||_2 by power iteration on M_b'M_b, one instance per workgroup ----
template <int NT, int LDSN>
__global__ __launch_bounds__(NT) void k_batch_norm(int count, int* queue, const int* order, const int* rowoff,
                                                   const int* coloff, const int* mrp,
                                                   const int* mcol, const double* mval,
                                                   const int* trp, const int* tcol,
                                                   const double* tval, const int* sel, double tol,
                                                   long long max_iter, double* v, double* w,
                                                   double* u, double* out)
{
    __shared__ double lds[2 * (NT / 64)];
    __shared__ double sbuf[LDSN];
    __shared__ int s_b;
    for (;;) {
        if (threadIdx.x == 0) s_b = atomicAdd(queue, 1);
        __syncthreads();
        int b = uniform_int(s_b);
        __syncthreads();
        if (b >= count) return;
        if (order != nullptr) b = uniform_int(order[b]);
        // every value that steers control flow around a barrier is moved to
        // scalar registers: a branch the compiler sees as divergent runs both
        // sides under an exec mask, and an empty-mask side whose loop is
        // steered by readfirstlane of idle lanes would execute a different
        // number of barriers in different waves
        const int c0 = uniform_int(coloff[b]), n = uniform_int(coloff[b + 1]) - c0;
        const int r0 = uniform_int(rowoff[b]), m = uniform_int(rowoff[b + 1]) - r0;
        const int nnz = uniform_int(mrp[r0 + m]) - uniform_int(mrp[r0]);
        const int skip = (sel != nullptr) ? (uniform_int(sel[b]) == 0) : 0;
        const int active = uniform_int((m > 0 && nnz > 0 && !skip) ? 1 : 0);
        double sig = 0.0;
        if (active) sig = power_norm_wg<NT, LDSN>(c0, n, r0, m, mrp, mcol, mval, trp, tcol, tval, tol, max_iter, v, w,
                                        u, lds, sbuf);
        if (threadIdx.x == 0) out[b] = sig;
        __syncthreads();
    }
}

// ||M_b||_2 of one instance by power iteration on M_b'M_b (the whole
// workgroup; every branch below is on workgroup-uniform values)
template <int NT, int LDSN>
__device__ double power_norm_wg(int c0, int n, int r0, int m, const int* mrp, const int* mcol,
                                const double* mval, const int* trp, const int* tcol, const double* tval,
                                double tol, long long max_iter, double* v, double* w, double* u, double* lds,
                                double* sbuf)
{
    // a small instance keeps v and w in LDS (the same values as the global
    // copies, gathered from LDS)
    const int stage = (n + m <= LDSN) ? 1 : 0;
    double* sv = sbuf;
    double* sw = sbuf + n;
    {
        // start vector: SplitMix64 of the local index (seed 0), in [-1, 1)
        double acc[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += NT) {
            unsigned long long z = (static_cast<unsigned long long>(j) + 1ull) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            const double val = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
            v[c0 + j] = val;
            acc[0] += val * val;
        }
        wg_reduce<1, 0u, NT>(acc, lds);
        const double nv = sqrt(acc[0]);
        for (int j = threadIdx.x; j < n; j += NT) {
            const double vj = v[c0 + j] / nv;
            v[c0 + j] = vj;
            if (stage) sv[j] = vj;
        }
        __syncthreads();
        double sig = 0.0, prev = 0.0;
        for (long long it = 1; it <= max_iter; ++it) {
            acc[0] = 0.0;
            for (int i = threadIdx.x; i < m; i += NT) {
                const double s = stage ? row_dot_lds<false>(mrp, Cols<false>{mcol, nullptr}, mval, nullptr, sv, c0, 0.0, r0 + i)
                                       : row_dot(mrp, Cols<false>{mcol, nullptr}, mval, v, r0 + i, c0);
                w[r0 + i] = s;
                if (stage) sw[i] = s;
                acc[0] += s * s;
            }
            wg_reduce<1, 0u, NT>(acc, lds);
            sig = sqrt(acc[0]);
            if (sig == 0.0) break;
            acc[0] = 0.0;
            for (int i = threadIdx.x; i < n; i += NT) {
                const double s = stage ? row_dot_lds<false>(trp, Cols<false>{tcol, nullptr}, tval, nullptr, sw, r0, 0.0, c0 + i)
                                       : row_dot(trp, Cols<false>{tcol, nullptr}, tval, w, c0 + i, r0);
                u[c0 + i] = s;
                acc[0] += s * s;
            }
            wg_reduce<1, 0u, NT>(acc, lds);
            const double nu = sqrt(acc[0]);
            if (nu == 0.0) break;
            for (int i = threadIdx.x; i < n; i += NT) {
                const double vi = u[c0 + i] / nu;
                v[c0 + i] = vi;
                if (stage) sv[i] = vi;
            }
            __syncthreads();
            if (fabs(sig - prev) <= tol * sig) break;
            prev = sig;
        }
        return sig;
    }
}

// ---- the solve -----------------------------------------------------------------

template <int NT, int LDSN, bool F32, bool C16>
__device__ __forceinline__ void batch_solve_one(const BatchDev& B, const BatchParams& P, int b, double* lds, double* sbuf)
{
    const Cols<C16> acol{B.acol, B.acol16}, tcol{B.tcol, B.tcol16}, qcol{B.qcol, B.qcol16};
    // per-instance values in scalar registers: the branches on them (closed
    // form vs inner solve, certificates) must be seen as uniform, or the
    // skipped side runs under an empty exec mask with its barrier count
    // steered by idle lanes
    const int v0 = uniform_int(B.voff[b]), n = uniform_int(B.voff[b + 1]) - v0;
    const int r0 = uniform_int(B.roff[b]), m = uniform_int(B.roff[b + 1]) - r0;
    const int tid = threadIdx.x;
    const unsigned long long t_start = wall_clock64();
    double* x = B.x + v0;   double* xa = B.xa + v0; double* xt = B.xt + v0;
    double* xbar = B.xbar;  double* aty = B.aty + v0; double* d = B.d + v0;
    const double* c = B.c + v0; const double* qd = B.qd + v0;
    const BoundAt lv{B.lv, v0}, uv{B.uv, v0};
    double* y = B.y + r0;   double* ya = B.ya + r0;  double* yt = B.yt;
    double* ytil = B.ytil;
    const double* lc = B.lc + r0; const double* uc = B.uc + r0;

    double* rhs = B.rhs + v0; double* g = B.g + v0; double* p = B.p + v0; double* hp = B.hp + v0;
    const double eta = uniform(B.eta[b]), omega0 = uniform(B.omega0[b]), normq = uniform(B.normq[b]);
    double omega = omega0, tau = eta / omega, sigma = eta * omega, it = 1.0 / tau;
    const int unb = uniform_int(B.unb[b]), qgen = uniform_int(B.qgen[b]);
    const double cmax = uniform(B.cmax[b]), bscale = uniform(B.bscale[b]), gammaq = uniform(B.gammaq[b]);
    double eps = INFINITY;
    long long inner_total = 0;

    // mixed precision: reference point (x_ref, y_ref) and its FP64 products
    // A x_ref (axref) and A' y_ref (aty, written by every check); zero until
    // the first check
    double* xref = B.xref; double* yref = B.yref; double* axref = B.axref + r0;
    // an instance small enough keeps the operands of its products in LDS:
    // sx (x_bar, written by the primal step) and sy (y, written by the dual
    // step), or their differences from the reference point in mixed
    // precision; with an inner solve also sp_ (its direction) and sxt (x_T)
    const int stage = (qgen ? 3 * n + m : n + m) <= LDSN ? 1 : 0;
    double* sx = sbuf;
    double* sy = sbuf + n;
    double* sp_ = sbuf + n + m;
    double* sxt = sbuf + 2 * n + m;
    // a closed-form instance small enough keeps its iterates in LDS for the
    // whole solve as well: x, its anchor, x_T, y and its anchor (x_T is
    // copied to HBM before each check, whose products read it there)
    const int stage2 = uniform_int((!qgen && 4 * n + 3 * m <= LDSN) ? 1 : 0);
    if (stage2) {
        x = sbuf + n + m;
        xa = x + n;
        xt = xa + n;
        y = xt + n;
        ya = y + m;
    }
    for (int i = tid; i < n; i += NT) {
        const double v = clampd(0.0, lv[i], uv[i]);
        x[i] = v; xa[i] = v; xt[i] = v;
        if constexpr (F32) { xref[v0 + i] = 0.0; aty[i] = 0.0; }
        if (stage && qgen) sxt[i] = v;
    }
    for (int j = tid; j < m; j += NT) {
        y[j] = 0.0; ya[j] = 0.0; yt[r0 + j] = 0.0;
        if constexpr (F32) { yref[r0 + j] = 0.0; axref[j] = 0.0; }
        if (stage) sy[j] = 0.0;
    }
    __syncthreads();

    long long k = 0, t = 0, restarts = 0;
    double R_start = 0.0, R_prev = 0.0, pid_int = 0.0, pid_prev = 0.0;
    int R_prev_valid = 0, status = 0;
    double ndx2 = 0.0, ndy2 = 0.0, ytil_max = 0.0, ptil_sum = 0.0, ptil_abs = 0.0, d_max = 0.0, cd = 0.0;
    double rp_ = 0.0, rd_ = 0.0, rg_ = 0.0, pobj = 0.0, dobj = 0.0;

    for (;;) {
        if ((k > 0 || P.max_iter == 0) && (k % P.check_every == 0 || k >= P.max_iter)) {
            if (stage2) {
                for (int i = tid; i < n; i += NT) B.xt[v0 + i] = xt[i];
                __syncthreads();
            }
            // ---- check at (x_T, y_T): KKT pieces and certificate pieces ----------
            double a[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) a[j] = 0.0;
            // max slots: 0 1 4 7 8 9 13 15, the rest sums
            constexpr unsigned kinds = (1u << 0) | (1u << 1) | (1u << 4) | (1u << 7) | (1u << 8) |
                                       (1u << 9) | (1u << 13) | (1u << 15);
            for (int i = tid; i < n; i += NT) {
                const double s = row_dot(B.trp, tcol, B.tval, yt, v0 + i, r0);
                aty[i] = s;
                a[0] = rcomb(R_MAX, a[0], fabs(s));
                if (k > 0) {
                    const double wv = row_dot(B.trp, tcol, B.tval, ytil, v0 + i, r0);
                    const double wh = projR(wv, lv[i], uv[i]);
                    a[1] = rcomb(R_MAX, a[1], fabs(wv - wh));
                    a[2] += supp(-wh, lv[i], uv[i]);
                    a[3] += supp_abs(-wh, lv[i], uv[i]);
                }
            }
            for (int j = tid; j < m; j += NT) {
                const double s = row_dot(B.arp, acol, B.aval, B.xt, r0 + j, v0);
                if constexpr (F32) axref[j] = s;
                a[4] = rcomb(R_MAX, a[4], fabs(s - clampd(s, lc[j], uc[j])));
                const double yj = yt[r0 + j];
                a[5] += supp(yj, lc[j], uc[j]);
                const double dv = yj - ya[j];
                a[6] += dv * dv;
                if (k > 0 && unb) {
                    const double ad = row_dot(B.arp, acol, B.aval, B.d, r0 + j, v0);
                    a[7] = rcomb(R_MAX, a[7], fabs(ad - projRec(ad, lc[j], uc[j])));
                }
            }
            __syncthreads();
            for (int i = tid; i < n; i += NT) {
                const double xi = xt[i], l = lv[i], u = uv[i];
                const double qx = qgen ? row_dot(B.qrp, qcol, B.qval, B.xt, v0 + i, v0) : qd[i] * xi;
                const double r = qx + c[i] + aty[i];
                const double rh = projR(r, l, u);
                a[8] = rcomb(R_MAX, a[8], fabs(r - rh));
                a[9] = rcomb(R_MAX, a[9], fabs(qx));
                a[10] += xi * qx;
                a[11] += c[i] * xi;
                a[12] += supp(-rh, l, u);
                a[13] = rcomb(R_MAX, a[13], fabs(xi - clampd(xi - r, l, u)));
                const double dv = xi - xa[i];
                a[14] += dv * dv;
                if (k > 0 && unb) {
                    const double qdv = qgen ? row_dot(B.qrp, qcol, B.qval, B.d, v0 + i, v0) : qd[i] * d[i];
                    a[15] = rcomb(R_MAX, a[15], fabs(qdv));
                }
            }
            if constexpr (F32) {
                // the new reference point: (x_T, y_T), whose products with A
                // and A' this check computed in FP64
                for (int i = tid; i < n; i += NT) xref[v0 + i] = xt[i];
                for (int j = tid; j < m; j += NT) yref[r0 + j] = yt[r0 + j];
            }
            wg_reduce<16, kinds, NT>(a, lds);
            rp_ = uniform(a[4] / bscale);
            double sd = a[9] > a[0] ? a[9] : a[0];
            sd = sd > cmax ? sd : cmax;
            rd_ = uniform(a[8] / (1.0 + sd));
            pobj = uniform(0.5 * a[10] + a[11]);
            const double dneg = 0.5 * a[10] + a[12] + a[5];
            dobj = uniform(-dneg);
            const double den = fabs(pobj) > fabs(dneg) ? fabs(pobj) : fabs(dneg);
            rg_ = uniform(fabs(a[10] + a[11] + a[12] + a[5]) / (1.0 + den));
            double worst = rp_ > rd_ ? rp_ : rd_;
            worst = worst > rg_ ? worst : rg_;
            bool pinf = false, dinf = false;
            if (k > 0 && ytil_max > 0.0 && isfinite(ytil_max)) {
                const double val = a[2] + ptil_sum;
                const double imp = val < 0.0 ? -val : 0.0;
                pinf = imp > 1e-9 * (a[3] + ptil_abs) && a[1] <= P.eps_inf * imp;
            }
            if (k > 0 && unb && d_max > 0.0 && isfinite(d_max) && cd / d_max < -P.tol) {
                const double v1 = a[7] / d_max, v2 = a[15] / d_max / gammaq;
                dinf = (v1 > v2 ? v1 : v2) <= P.eps_inf;
            }
            int restart = 0;
            if (!isfinite(worst) || worst != worst) status = 5;
            else if (worst <= P.tol) status = 1;
            else if (pinf) status = 2;
            else if (dinf) status = 3;
            else if (k >= P.max_iter) status = 4;
            else {
                const double R = sqrt(omega * ndx2 + ndy2 / omega);
                restart = R <= P.rs_suff * R_start ||
                          (R_prev_valid && R <= P.rs_nec * R_start && R > R_prev) ||
                          (double)t >= P.rs_art * (double)k;
                R_prev = uniform(R);
                R_prev_valid = 1;
                if (restart) {
                    const double mx = sqrt(a[14]), my = sqrt(a[6]);
                    if (mx > 1e-10 && my > 1e-10 && isfinite(mx) && isfinite(my)) {
                        const double so = sqrt(omega);
                        const double e = log(so * mx / (my / so));
                        pid_int = uniform(pid_int + e);
                        double lw = log(omega) - (P.kp * e + P.ki * pid_int + P.kd * (e - pid_prev));
                        const double lo = log(omega0) - 10.0, hi = log(omega0) + 10.0;
                        lw = lw < lo ? lo : (lw > hi ? hi : lw);
                        omega = uniform(exp(lw));
                        pid_prev = uniform(e);
                    }
                    tau = uniform(eta / omega);
                    sigma = uniform(eta * omega);
                    it = uniform(1.0 / tau);
                    t = 0;
                    R_prev_valid = 0;
                    ++restarts;
                }
            }
            if (status) break;
            if (restart) {
                for (int i = tid; i < n; i += NT) { x[i] = xt[i]; xa[i] = xt[i]; }
                for (int j = tid; j < m; j += NT) { y[j] = yt[r0 + j]; ya[j] = yt[r0 + j]; }
            }
            if (stage) {
                // y after a restart, and (mixed) its difference from the new reference
                for (int j = tid; j < m; j += NT) {
                    if constexpr (F32) sy[j] = y[j] - yref[r0 + j];
                    else sy[j] = y[j];
                }
            }
            __syncthreads();
        }
        if (k >= P.max_iter) { status = 4; break; }
        const bool store = ((k + 1) % P.check_every == 0) || (k + 1 >= P.max_iter);

        if (!qgen) {
            // ---- primal step: closed form (Section 2.2) and x_bar -----------------
            for (int i = tid; i < n; i += NT) {
                const double s =
                    stage ? row_dot_lds<F32>(B.trp, tcol, B.tval, B.tval32, sy, r0, aty[i], v0 + i)
                          : row_dot_bulk<F32>(B.trp, tcol, B.tval, B.tval32, B.y, yref, aty[i], v0 + i, r0);
                const double xi = x[i];
                const double v = clampd((xi * it - c[i] - s) / (qd[i] + it), lv[i], uv[i]);
                xt[i] = v;
                const double xb = 2.0 * v - xi;
                if (!stage) xbar[v0 + i] = xb;   // staged: the dual step reads sx
                if (stage) {
                    if constexpr (F32) sx[i] = xb - xref[v0 + i];
                    else sx[i] = xb;
                }
            }
            __syncthreads();
        } else {
            // ---- primal step: boxed CG (MPRGP) on 1/2 x'(Q + I/tau)x - rhs'x -----
            const double abar = P.abar_scale / (normq + it);
            double st[3] = {0.0, 0.0, 0.0};   // ||g^P||^2, ||beta||^2, phit'phi
            for (int i = tid; i < n; i += NT) {
                const double aty_i =
                    stage ? row_dot_lds<F32>(B.trp, tcol, B.tval, B.tval32, sy, r0, aty[i], v0 + i)
                          : row_dot_bulk<F32>(B.trp, tcol, B.tval, B.tval32, B.y, yref, aty[i], v0 + i, r0);
                const double r = x[i] * it - c[i] - aty_i;
                rhs[i] = r;
                const double xi = xt[i];
                const double qx = stage ? row_dot_lds<false>(B.qrp, qcol, B.qval, nullptr, sxt, v0, 0.0, v0 + i)
                                        : row_dot(B.qrp, qcol, B.qval, B.xt, v0 + i, v0);
                const double gi = qx + it * xi - r;
                g[i] = gi;
                const Split sp = split(xi, gi, lv[i], uv[i], abar);
                st[0] += sp.phi * sp.phi + sp.beta * sp.beta;
                st[1] += sp.beta * sp.beta;
                st[2] += sp.phit * sp.phi;
            }
            wg_reduce<3, 0u, NT>(st, lds);
            if (isinf(eps) && P.eps_fixed <= 0.0) eps = uniform(fmax(P.gamma_inner * sqrt(st[0]), P.eps_min));
            const double eps_use = P.eps_fixed > 0.0 ? P.eps_fixed : eps;
            long long inner = 0;
            int last = STEP_NONE;
            double gam = 0.0;
            bool done = sqrt(st[0]) <= eps_use || P.max_inner <= 0;
            int mode = (st[1] <= P.mprgp_gamma * P.mprgp_gamma * st[2]) ? DIR_PHI : DIR_BETA;
            while (!done) {
                for (int i = tid; i < n; i += NT) {
                    const Split sp = split(xt[i], g[i], lv[i], uv[i], abar);
                    const double pn = mode == DIR_BETA ? sp.beta : (mode == DIR_PHI ? sp.phi : sp.phi - gam * p[i]);
                    p[i] = pn;
                    if (stage) sp_[i] = pn;
                }
                __syncthreads();
                double hs[3] = {0.0, 0.0, INFINITY};   // p'Hp, g'p, feasible step
                for (int i = tid; i < n; i += NT) {
                    const double pi = p[i], xi = xt[i];
                    const double h =
                        (stage ? row_dot_lds<F32>(B.qrp, qcol, B.qval, B.qval32, sp_, v0, 0.0, v0 + i)
                               : hp_dot<F32>(B.qrp, qcol, B.qval, B.qval32, B.p, v0 + i, v0)) + it * pi;
                    hp[i] = h;
                    hs[0] += pi * h;
                    hs[1] += g[i] * pi;
                    double fs = INFINITY;
                    if (pi > 0.0 && isfinite(lv[i])) fs = (xi - lv[i]) / pi;
                    else if (pi < 0.0 && isfinite(uv[i])) fs = (xi - uv[i]) / pi;
                    hs[2] = fmin(hs[2], fs);
                }
                wg_reduce_min3<NT>(hs, lds);
                if (!(hs[0] > 0.0)) break;
                const double af = hs[2] < 0.0 ? 0.0 : hs[2];
                const double acg = hs[1] / hs[0];
                int kind;
                double alpha;
                if (mode == DIR_BETA) { kind = STEP_PROP; alpha = acg < af ? acg : af; }
                else if (acg <= af) { kind = STEP_CG; alpha = acg; }
                else { kind = STEP_EXPAND; alpha = af; }
                double us[4] = {0.0, 0.0, 0.0, 0.0};   // stats and phi'Hp
                for (int i = tid; i < n; i += NT) {
                    const double l = lv[i], u = uv[i];
                    double xi = clampd(xt[i] - alpha * p[i], l, u);
                    const double gi = g[i] - alpha * hp[i];
                    g[i] = gi;
                    const Split sp = split(xi, gi, l, u, abar);
                    if (kind == STEP_EXPAND) {
                        xi = clampd(xi - abar * sp.phi, l, u);
                    } else {
                        us[0] += sp.phi * sp.phi + sp.beta * sp.beta;
                        us[1] += sp.beta * sp.beta;
                        us[2] += sp.phit * sp.phi;
                        us[3] += sp.phi * hp[i];
                    }
                    xt[i] = xi;
                    if (stage) sxt[i] = xi;
                }
                ++inner;
                if (kind == STEP_EXPAND) {
                    __syncthreads();
                    us[0] = us[1] = us[2] = 0.0;
                    for (int i = tid; i < n; i += NT) {
                        const double xi = xt[i];
                        const double qx = stage ? row_dot_lds<false>(B.qrp, qcol, B.qval, nullptr, sxt, v0, 0.0, v0 + i)
                                                : row_dot(B.qrp, qcol, B.qval, B.xt, v0 + i, v0);
                        const double gi = qx + it * xi - rhs[i];
                        g[i] = gi;
                        const Split sp = split(xi, gi, lv[i], uv[i], abar);
                        us[0] += sp.phi * sp.phi + sp.beta * sp.beta;
                        us[1] += sp.beta * sp.beta;
                        us[2] += sp.phit * sp.phi;
                    }
                }
                wg_reduce<4, 0u, NT>(us, lds);
                if (kind == STEP_CG) gam = us[3] / hs[0];
                last = kind;
                done = sqrt(us[0]) <= eps_use || inner >= P.max_inner;
                const bool prop = us[1] <= P.mprgp_gamma * P.mprgp_gamma * us[2];
                mode = !prop ? DIR_BETA : (last == STEP_CG ? DIR_CONJ : DIR_PHI);
            }
            inner_total += inner;
            for (int i = tid; i < n; i += NT) {
                const double xb = 2.0 * xt[i] - x[i];
                if (!stage) xbar[v0 + i] = xb;
                if (stage) {
                    if constexpr (F32) sx[i] = xb - xref[v0 + i];
                    else sx[i] = xb;
                }
            }
            __syncthreads();
        }
        // ---- dual step and Halpern on y --------------------------------------------
        const double w = (double)(t + 1) / (double)(t + 2), wa = 1.0 / (double)(t + 2);
        const double th = P.theta;
        double a[7] = {0, 0, 0, 0, 0, 0, 0};
        constexpr unsigned kinds7 = (1u << 2) | (1u << 5);   // max slots, the rest sums
        for (int j = tid; j < m; j += NT) {
            const double s =
                stage ? row_dot_lds<F32>(B.arp, acol, B.aval, B.aval32, sx, v0, axref[j], r0 + j)
                      : row_dot_bulk<F32>(B.arp, acol, B.aval, B.aval32, xbar, xref, axref[j], r0 + j, v0);
            const double yj = y[j], l = lc[j], u = uc[j];
            const double v = yj / sigma + s;
            const double ytj = sigma * (v - clampd(v, l, u));
            const double dy = ytj - yj;
            a[1] += dy * dy;
            if (store) yt[r0 + j] = ytj;   // read only by the check that follows
            const double yn = P.use_halpern ? w * ((1.0 + th) * ytj - th * yj) + wa * ya[j] : ytj;
            y[j] = yn;
            if (stage) {
                if constexpr (F32) sy[j] = yn - yref[r0 + j];
                else sy[j] = yn;
            }
            if (store) {
                const double yy = projY(dy, l, u);
                ytil[r0 + j] = yy;
                a[2] = rcomb(R_MAX, a[2], fabs(yy));
                a[3] += supp(yy, l, u);
                a[4] += supp_abs(yy, l, u);
            }
        }
        // ---- Halpern on x ---------------------------------------------------------
        for (int i = tid; i < n; i += NT) {
            const double xti = xt[i], xi = x[i];
            const double dx = xti - xi;
            a[0] += dx * dx;
            x[i] = P.use_halpern ? w * ((1.0 + th) * xti - th * xi) + wa * xa[i] : xti;
            if (store && unb) {
                const double di = projRec(dx, lv[i], uv[i]);
                d[i] = di;
                a[5] = rcomb(R_MAX, a[5], fabs(di));
                a[6] += c[i] * di;
            }
        }
        wg_reduce<7, kinds7, NT>(a, lds);
        ndx2 = uniform(a[0]);
        ndy2 = uniform(a[1]);
        if (P.eps_fixed <= 0.0) eps = uniform(fmin(eps, fmax(P.gamma_inner * omega * sqrt(ndx2) / tau, P.eps_min)));
        if (store) {
            ytil_max = uniform(a[2]); ptil_sum = uniform(a[3]); ptil_abs = uniform(a[4]);
            d_max = uniform(unb ? a[5] : 0.0);
            cd = uniform(unb ? a[6] : 0.0);
        }
        ++k;
        ++t;
        if (t == 1) R_start = uniform(sqrt(omega * ndx2 + ndy2 / omega));
    }
    if (tid == 0) {
        BatchOut o;
        o.status = status;
        o.pad = 0;
        o.iterations = k;
        o.restarts = restarts;
        o.inner_iterations = inner_total;
        o.r_primal = rp_; o.r_dual = rd_; o.r_gap = rg_;
        o.pobj = pobj; o.dobj = dobj; o.omega = omega;
        o.ytil_max = ytil_max; o.d_max = d_max;
        o.t_start = t_start;
        o.t_end = wall_clock64();
        B.out[b] = o;
    }
    __syncthreads();
}

// WPE: waves per SIMD the register allocation must allow (1: no limit
// beyond the workgroup size; more trades spills for resident instances)
template <int NT, int LDSN, int WPE, bool F32, bool C16>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_batch_solve(BatchDev B, BatchParams P)
{
    __shared__ double lds[16 * (NT / 64)];
    __shared__ double sbuf[LDSN];
    __shared__ int s_b;
    for (;;) {
        if (threadIdx.x == 0) s_b = atomicAdd(B.queue, 1);
        __syncthreads();
        int b = uniform_int(s_b);
        __syncthreads();
        if (b >= B.count) return;
        if (B.order != nullptr) b = uniform_int(B.order[b]);
        batch_solve_one<NT, LDSN, F32, C16>(B, P, b, lds, sbuf);
    }
}

// ---- launch shapes ---------------------------------------------------------------
// (threads per workgroup, LDS doubles for staged operands): more threads per
// instance against more instances resident per CU; which wins depends on the
// instance sizes, so the host can time them on a batch (the autotuner) or use
// the default.

template <int NT, int LDSN, int WPE, bool F32>
hipError_t solve_shape(const BatchDev& B, const BatchParams& P, int grid, hipStream_t s)
{
    if (B.acol16) k_batch_solve<NT, LDSN, WPE, F32, true><<<grid, NT, 0, s>>>(B, P);
    else k_batch_solve<NT, LDSN, WPE, F32, false><<<grid, NT, 0, s>>>(B, P);
    return hipGetLastError();
}

template <int NT, int LDSN, int WPE>
hipError_t norm_shape(const BatchDev& B, const int* rowoff, const int* coloff, const int* mrp,
                      const int* mcol, const double* mval, const int* trp, const int* tcol,
                      const double* tval, const int* sel, double tol, long long max_iter, double* v,
                      double* w, double* u, double* out, int grid, hipStream_t s)
{
    k_batch_norm<NT, LDSN><<<grid, NT, 0, s>>>(B.count, B.queue, B.order, rowoff, coloff, mrp, mcol, mval,
                                               trp, tcol, tval, sel, tol, max_iter, v, w, u, out);
    return hipGetLastError();
}

template <int NT, int LDSN, int WPE>
int resident_per_cu(int which)
{
    int nb = 0;
    hipError_t e;
    if (which == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_solve<NT, LDSN, WPE, false, true>, NT, 0);
    else if (which == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_solve<NT, LDSN, WPE, true, true>, NT, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_norm<NT, LDSN>, NT, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

#define PDHCG_BATCH_SHAPES(X) \
    X(512, 8192, 1) X(256, 6144, 1) X(256, 2048, 1) X(256, 2048, 4) X(128, 1536, 1) X(128, 1536, 4) X(64, 1536, 1) \
    X(64, 1024, 4) X(1024, 12288, 1) X(256, 3072, 4) X(256, 3840, 4) X(256, 4608, 4) X(256, 4992, 4)

const BatchShape* batch_shapes(int* count)
{
#define PDHCG_SHAPE_ENTRY(T_, L_, W_) {T_, L_, W_},
    static const BatchShape tab[] = {PDHCG_BATCH_SHAPES(PDHCG_SHAPE_ENTRY)};
#undef PDHCG_SHAPE_ENTRY
    *count = (int)(sizeof(tab) / sizeof(tab[0]));
    return tab;
}

// persistent grid of a shape: the workgroups one pass of the device holds
// (occupancy x CUs), at most one per instance; which: 0 FP64 solve, 1 mixed
// solve, 2 norm kernel
int batch_grid(int shape, int which, int count)
{
    static const int cus = [] {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
            return c;
        return 256;
    }();
    static std::atomic<int> occ[16][3];   // resident workgroups per CU, 0 = not asked yet
    if (shape < 0 || shape >= 16 || which < 0 || which > 2) return 1;
    int per = occ[shape][which].load(std::memory_order_relaxed);
    if (per == 0) {
        int k = 0;
#define PDHCG_SHAPE_OCC(T_, L_, W_) if (k++ == shape) per = resident_per_cu<T_, L_, W_>(which);
        PDHCG_BATCH_SHAPES(PDHCG_SHAPE_OCC)
#undef PDHCG_SHAPE_OCC
        if (per < 1) per = 1;
        occ[shape][which].store(per, std::memory_order_relaxed);
    }
    const long long g = (long long)per * cus;
    const long long r = count < g ? count : g;
    return r < 1 ? 1 : (int)r;
}

hipError_t launch_batch_norm(const BatchDev& B, int shape, const int* rowoff, const int* coloff,
                             const int* mrp, const int* mcol, const double* mval,
                             const int* trp, const int* tcol, const double* tval, const int* sel,
                             double tol, long long max_iter, double* v, double* w, double* u,
                             double* out, hipStream_t s)
{
    const int grid = batch_grid(shape, 2, B.count);
    int k = 0;
#define PDHCG_SHAPE_NORM(T_, L_, W_) \
    if (k++ == shape) return norm_shape<T_, L_, W_>(B, rowoff, coloff, mrp, mcol, mval, trp, tcol, tval, sel, tol, max_iter, v, w, u, out, grid, s);
    PDHCG_BATCH_SHAPES(PDHCG_SHAPE_NORM)
#undef PDHCG_SHAPE_NORM
    return hipErrorInvalidValue;
}

hipError_t launch_batch_solve(const BatchDev& B, const BatchParams& P, int shape, hipStream_t s)
{
    const bool f32 = B.aval32 != nullptr;
    const int grid = batch_grid(shape, f32 ? 1 : 0, B.count);
    int k = 0;
#define PDHCG_SHAPE_SOLVE(T_, L_, W_) \
    if (k++ == shape) return f32 ? solve_shape<T_, L_, W_, true>(B, P, grid, s) : solve_shape<T_, L_, W_, false>(B, P, grid, s);
    PDHCG_BATCH_SHAPES(PDHCG_SHAPE_SOLVE)
#undef PDHCG_SHAPE_SOLVE
    return hipErrorInvalidValue;
}

}  // namespace pdhcg
