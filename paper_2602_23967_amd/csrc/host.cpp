// host.cpp -- C ABI of the gfx950 PDHCG-II solver: input validation, device
// setup (transpose, SpMV schedules, norm estimates) and the host side of the
// solve loop.  All arithmetic of the method runs in kernels.hip; the host
// only enqueues kernels, watches a pinned status word the kernels post, and
// copies results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/pdhcg.h"
#include "host_internal.h"
#include "pdhcg_internal.h"

using namespace pdhcg;

namespace {

struct EventPair {
    hipEvent_t ev[2];   // around the main kernel of one launch (not its finishing kernel)
    int fam;
};

}  // namespace

struct qp_handle {
    int64_t n = 0, m = 0;
    DevState S;
    hipStream_t own = nullptr, stream = nullptr;
    unsigned long long* hstat = nullptr;
    unsigned long long* hcheck = nullptr;
    std::vector<void*> dev_allocs;
    int solved = 0;
    int status = QP_NOT_SOLVED;
    qp_info info{};
    double norm_A = 0.0, norm_Q_raw = 0.0, norm_Q = 0.0, omega0 = 1.0;
    double c_max = 0.0, bscale_p = 1.0, gamma_q = 1.0;
    int has_unbounded_x = 0;
    int qkind = 0;   // 0 none, 1 diagonal, 2 general
    double setup_seconds = 0.0;
    // timing
    std::vector<EventPair> ev_pool;
    size_t ev_used = 0;
    int timing = 0;
    int64_t fam_launches[QP_NFAM] = {};
    // FP32 copies of the matrix values, made at the first mixed-precision solve
    float *val32_A = nullptr, *val32_AT = nullptr, *val32_Q = nullptr, *val32_R = nullptr;
    // graph of `graph_steps` inner steps (captured once per precision)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_steps = 0, graph_mixed = -1;
};

namespace {

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(QP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

// A copy ordered on `s` that has completed when the call returns.  Every
// copy of the library goes through a stream of its own handle (created
// non-blocking), never the null stream, so one handle's copies do not wait
// for the work of other handles in flight on the device.
hipError_t copy_wait(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Device memory comes from the stream-ordered allocator on the handle's own
// stream (and goes back the same way), so creating and destroying handles
// does not synchronise the device.
template <class T>
int dalloc(qp_handle* h, T** p, size_t count)
{
    void* q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMallocAsync(&q, bytes, h->own);
    if (e != hipSuccess) return fail(QP_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    h->dev_allocs.push_back(q);
    *p = static_cast<T*>(q);
    return 0;
}

// the bulk products (not the checks) read FP32 values when the solve is in
// mixed precision; the copies are made once and kept for later solves
int set_precision(qp_handle* h, int precision)
{
    DevState& S = h->S;
    if (precision == QP_PRECISION_MIXED) {
        struct Item { CsrDev* M; float** keep; } items[4] = {{&S.A, &h->val32_A}, {&S.AT, &h->val32_AT},
                                                            {&S.Q, &h->val32_Q}, {&S.R, &h->val32_R}};
        for (Item& it : items) {
            if (it.M->nnz == 0 || !it.M->val) continue;
            if (!*it.keep) {
                if (int rc = dalloc(h, it.keep, (size_t)it.M->nnz)) return rc;
                HIPCHK(launch_to_f32(it.M->val, *it.keep, it.M->nnz, h->stream));
            }
            it.M->val32 = *it.keep;
        }
    } else {
        S.A.val32 = S.AT.val32 = S.Q.val32 = S.R.val32 = nullptr;
    }
    S.mixed = precision == QP_PRECISION_MIXED;
    if (S.mixed && !S.xref) {
        int rc;
        if ((rc = dalloc(h, &S.xref, (size_t)h->n)) || (rc = dalloc(h, &S.atyref, (size_t)h->n)) ||
            (rc = dalloc(h, &S.yref, (size_t)h->m)) || (rc = dalloc(h, &S.axref, (size_t)h->m)) ||
            (rc = dalloc(h, &S.dxb32, (size_t)h->n)) || (rc = dalloc(h, &S.dy32, (size_t)h->m)))
            return rc;
    }
    return 0;
}

template <class T>
int upload(qp_handle* h, T** p, const T* src, size_t count)
{
    int rc = dalloc(h, p, count);
    if (rc) return rc;
    if (count) HIPCHK(copy_wait(*p, src, count * sizeof(T), hipMemcpyHostToDevice, h->own));
    return 0;
}

int upload_bounds(qp_handle* h, DevState& S, const std::vector<double>& lv, const std::vector<double>& uv)
{
    std::vector<unsigned char> cls;
    std::vector<double> tl, tu;
    const int mode = classify_bounds(lv, uv, cls, tl, tu);
    S.lv = BoundVec{};
    S.uv = BoundVec{};
    S.lv.mode = S.uv.mode = mode;
    int rc;
    if (mode == 1) {
        S.lv.k = tl[0];
        S.uv.k = tu[0];
    } else if (mode == 2) {
        unsigned char* dc = nullptr;
        double *dl = nullptr, *du = nullptr;
        if ((rc = upload(h, &dc, cls.data(), cls.size())) || (rc = upload(h, &dl, tl.data(), tl.size())) ||
            (rc = upload(h, &du, tu.data(), tu.size())))
            return rc;
        S.lv.cls = S.uv.cls = dc;
        S.lv.tab = dl;
        S.uv.tab = du;
    } else {
        double *dl = nullptr, *du = nullptr;
        if ((rc = upload(h, &dl, lv.data(), lv.size())) || (rc = upload(h, &du, uv.data(), uv.size()))) return rc;
        S.lv.a = dl;
        S.uv.a = du;
    }
    return 0;
}

int upload_csr(qp_handle* h, CsrDev& M, int64_t rows, int64_t cols, const int64_t* rp,
               const int32_t* cj, const double* v)
{
    M.rows = (int)rows;
    M.cols = (int)cols;
    M.nnz = rp ? rp[rows] : 0;
    if (rp && cols >= PART_MIN_COLS && rows > 0 && M.nnz > 0 && M.nnz >= (int64_t)PART_MIN_NNZ_ROW * rows) {
        std::vector<int> prow;
        std::vector<int32_t> pcol;
        std::vector<double> pval;
        std::vector<BlkDesc> blk;
        if (build_parts(rows, cols, rp, cj, v, prow, pcol, pval, blk)) {
            int rc;
            M.nparts = NPARTS;
            M.nblk = (int)blk.size();
            if ((rc = upload(h, &M.rowptr, prow.data(), prow.size()))) return rc;
            if ((rc = upload(h, &M.col, pcol.data(), pcol.size()))) return rc;
            if ((rc = upload(h, &M.val, pval.data(), pval.size()))) return rc;
            if ((rc = upload(h, &M.blk, blk.data(), blk.size()))) return rc;
            if ((rc = dalloc(h, &M.ypart, (size_t)NPARTS * rows))) return rc;
            if ((rc = dalloc(h, &M.seg_part, 1))) return rc;
            if ((rc = dalloc(h, &M.lr_info, 1))) return rc;
            M.nlr = 0;
            return 0;
        }
    }
    std::vector<int> rp32(rows + 1, 0);
    for (int64_t i = 0; i <= rows; ++i) rp32[i] = rp ? (int)rp[i] : 0;
    int rc;
    if ((rc = upload(h, &M.rowptr, rp32.data(), rows + 1))) return rc;
    if ((rc = upload(h, &M.col, cj, (size_t)M.nnz))) return rc;
    if ((rc = upload(h, &M.val, v, (size_t)M.nnz))) return rc;
    std::vector<int64_t> rp64(rows + 1, 0);
    if (rp) std::copy(rp, rp + rows + 1, rp64.begin());
    std::vector<BlkDesc> blk;
    int nlr = 0, nseg = 0;
    build_plan(rows, rp64.data(), blk, nlr, nseg);
    M.nblk = (int)blk.size();
    if ((rc = upload(h, &M.blk, blk.data(), blk.size()))) return rc;
    if ((rc = dalloc(h, &M.seg_part, (size_t)std::max(nseg, 1)))) return rc;
    // long rows: those the finishing kernel sums with the whole block first
    // (all when they are few, else the ones with many segments), then the
    // rest, each group in row order
    std::vector<int> info;
    int ncoop = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (const BlkDesc& b : blk)
            if (b.nrows == 0 && b.nseg > 0 && b.seg == 0) {
                const bool coop = nlr <= LR_COOP || b.nseg > LR_SEG_SERIAL;
                if (coop != (pass == 0)) continue;
                info.push_back(b.row0);
                info.push_back(b.seg_base);
                info.push_back(b.nseg);
                ncoop += coop ? 1 : 0;
            }
    M.nlr = nlr;
    M.nlr_coop = ncoop;
    if (nlr > 0) std::copy(info.begin(), info.begin() + 3, M.lr0);
    if ((rc = upload(h, &M.lr_info, info.data(), info.size()))) return rc;
    return 0;
}

hipStream_t stream_of(const qp_handle* h) { return h->stream; }

// power-iteration estimate of ||M||_2 through M'M (Mt = M' as a CSR),
// the same sequence as the oracle: w = M v, sigma = ||w||, u = M' w,
// v = u / ||u||, stop when sigma changes by <= tol * sigma
// ||M||_2 by power iteration on M'M.  is_q: M is the (symmetric) Q operator,
// applied as [P | R'] on [v; R v] when Q is factored.
int power_norm(qp_handle* h, const CsrDev& M, const CsrDev& Mt, double tol, int64_t max_iter,
               double* out, bool is_q = false)
{
    *out = 0.0;
    if (M.rows == 0 || M.cols == 0 || M.nnz == 0) return 0;
    DevState& S = h->S;
    hipStream_t s = stream_of(h);
    double* v = S.v1;
    double* w = S.v2;
    const int cols = is_q ? S.n : M.cols;
    HIPCHK(launch_power_start(S, v, cols, s));
    HIPCHK(launch_scale(S, v, cols, s));
    double sig = 0.0, prev = 0.0;
    for (int64_t it = 1; it <= max_iter; ++it) {
        if (is_q) HIPCHK(launch_tail(S, v, v + S.n, false, s));
        HIPCHK(launch_spmv_norm(S, M, v, w, s));
        HIPCHK(hipMemcpyAsync(&h->hcheck[1], &S.ctrl->pw_norm, sizeof(double), hipMemcpyDeviceToHost, s));
        if (is_q) HIPCHK(launch_tail(S, w, w + S.n, false, s));
        HIPCHK(launch_spmv_norm(S, Mt, w, v, s));
        HIPCHK(hipMemcpyAsync(&h->hcheck[2], &S.ctrl->pw_norm, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(launch_scale(S, v, cols, s));
        HIPCHK(hipStreamSynchronize(s));
        double nu;
        std::memcpy(&sig, &h->hcheck[1], sizeof(double));
        std::memcpy(&nu, &h->hcheck[2], sizeof(double));
        if (sig == 0.0 || nu == 0.0) break;
        if (std::fabs(sig - prev) <= tol * sig) break;
        prev = sig;
    }
    *out = sig;
    return 0;
}

// Q is either given as one CSR (k == 0) or as P (in Qp/Qj/Qv, may be NULL)
// plus R'R with R k x n CSR.
int create_impl(int64_t n, int64_t m, const int64_t* Qp, const int32_t* Qj, const double* Qv,
                const int64_t* Ap, const int32_t* Aj, const double* Av, const double* c,
                const double* lc, const double* uc, const double* lb, const double* ub,
                qp_handle** out, int64_t k = 0, const int64_t* Rp = nullptr,
                const int32_t* Rj = nullptr, const double* Rv = nullptr)
{
    const double t0 = now_s();
    int rc;
    std::vector<double> lvv(n), uvv(n);
    for (int64_t i = 0; i < n; ++i) {
        lvv[i] = lb ? lb[i] : -INFINITY;
        uvv[i] = ub ? ub[i] : INFINITY;
    }
    if ((rc = check_bounds("lb/ub", n, lvv.data(), uvv.data()))) return rc;
    if ((rc = check_vec("c", n, c, false))) return rc;
    std::vector<int64_t> a_empty(1, 0);
    if (!Ap) {
        if (m != 0) return fail(QP_ERR_INVALID_ARG, "A: row pointer is NULL");
        Ap = a_empty.data();
    }
    if ((rc = check_csr("A", m, n, Ap, Aj, Av))) return rc;
    if (Qp) {
        if ((rc = check_csr("Q", n, n, Qp, Qj, Qv))) return rc;
        if ((rc = check_symmetric(n, Qp, Qj, Qv))) return rc;
    }
    if (k < 0 || k >= INT32_MAX || n + k >= INT32_MAX) return fail(QP_ERR_INVALID_ARG, "bad factor rank k");
    if (k > 0) {
        if (!Rp) return fail(QP_ERR_INVALID_ARG, "R: row pointer is NULL");
        if ((rc = check_csr("R", k, n, Rp, Rj, Rv))) return rc;
    }

    // ---- device setup -------------------------------------------------------
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(QP_ERR_DEVICE, "no HIP device available");

    qp_handle* h = new qp_handle();
    h->n = n;
    h->m = m;
    DevState& S = h->S;
    S.n = (int)n;
    S.m = (int)m;
    auto bail = [&](int code) {
        qp_destroy(h);
        return code;
    };
    if (hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipStreamCreate failed"));
    h->stream = h->own;
    if (hipHostMalloc((void**)&h->hstat, 4 * sizeof(unsigned long long),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipHostMalloc failed"));
    h->hcheck = h->hstat + 1;
    std::memset(h->hstat, 0, 4 * sizeof(unsigned long long));
    if (hipHostGetDevicePointer((void**)&S.dstat, h->hstat, 0) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipHostGetDevicePointer failed"));
    S.dcheck = S.dstat + 1;

    // Q kind: none, diagonal (closed-form primal step) or general
    std::vector<double> qd(n, 0.0);
    h->qkind = 0;
    // factored Q: the product matrix [P | R'] (n x (n + k)) and R
    std::vector<int64_t> mp, rtp;
    std::vector<int32_t> mj, rtj;
    std::vector<double> mv, rtv;
    if (k > 0) {
        transpose(k, n, Rp, Rj, Rv, rtp, rtj, rtv);
        mp.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            mp[i + 1] = mp[i] + (Qp ? Qp[i + 1] - Qp[i] : 0) + (rtp[i + 1] - rtp[i]);
        mj.resize(mp[n]);
        mv.resize(mp[n]);
        for (int64_t i = 0; i < n; ++i) {
            int64_t q = mp[i];
            if (Qp)
                for (int64_t e = Qp[i]; e < Qp[i + 1]; ++e) { mj[q] = Qj[e]; mv[q] = Qv[e]; ++q; }
            for (int64_t e = rtp[i]; e < rtp[i + 1]; ++e) { mj[q] = (int32_t)(n + rtj[e]); mv[q] = rtv[e]; ++q; }
        }
        if (mp[n] >= INT32_MAX) return bail(fail(QP_ERR_INVALID_ARG, "too many nonzeros in [P | R']"));
        h->qkind = 2;
        S.k = (int)k;
    } else if (Qp) {
        h->qkind = 1;
        for (int64_t i = 0; i < n && h->qkind == 1; ++i)
            for (int64_t k = Qp[i]; k < Qp[i + 1]; ++k)
                if (Qj[k] != i) { h->qkind = 2; break; }
        if (h->qkind == 1)
            for (int64_t i = 0; i < n; ++i)
                for (int64_t k = Qp[i]; k < Qp[i + 1]; ++k) qd[i] += Qv[k];
    }
    S.qdiag = h->qkind < 2;

    std::vector<int64_t> tp;
    std::vector<int32_t> tj;
    std::vector<double> tv;
    transpose(m, n, Ap, Aj, Av, tp, tj, tv);
    if ((rc = upload_csr(h, S.A, m, n, Ap, Aj, Av))) return bail(rc);
    if ((rc = upload_csr(h, S.AT, n, m, tp.data(), tj.data(), tv.data()))) return bail(rc);
    std::vector<int64_t> q_empty(n + 1, 0);
    if (k > 0) {
        if ((rc = upload_csr(h, S.Q, n, n + k, mp.data(), mj.data(), mv.data()))) return bail(rc);
        if ((rc = upload_csr(h, S.R, k, n, Rp, Rj, Rv))) return bail(rc);
    } else {
        if ((rc = upload_csr(h, S.Q, n, n, Qp ? Qp : q_empty.data(), Qj, Qv))) return bail(rc);
    }

    std::vector<double> lcv(m), ucv(m);
    for (int64_t i = 0; i < m; ++i) { lcv[i] = lc[i]; ucv[i] = uc[i]; }
    if ((rc = upload(h, &S.qd, qd.data(), n))) return bail(rc);
    if ((rc = upload(h, &S.c, c, n))) return bail(rc);
    if ((rc = upload_bounds(h, S, lvv, uvv))) return bail(rc);
    if ((rc = upload(h, &S.lc, lcv.data(), m))) return bail(rc);
    if ((rc = upload(h, &S.uc, ucv.data(), m))) return bail(rc);
    double** nvecs[] = {&S.x, &S.xa, &S.rhs, &S.g, &S.hp, &S.aty, &S.xbar};
    for (double** pv : nvecs)
        if ((rc = dalloc(h, pv, n))) return bail(rc);
    double** tvecs[] = {&S.xt, &S.p, &S.dx};   // operands of Q: room for R times them
    for (double** pv : tvecs)
        if ((rc = dalloc(h, pv, n + k))) return bail(rc);
    double** mvecs[] = {&S.y, &S.ya, &S.yt, &S.ytil};
    for (double** pv : mvecs)
        if ((rc = dalloc(h, pv, m))) return bail(rc);
    const int64_t nm = std::max(n, m) + k;
    if ((rc = dalloc(h, &S.v1, nm))) return bail(rc);
    if ((rc = dalloc(h, &S.v2, nm))) return bail(rc);
    if ((rc = dalloc(h, &S.ctrl, 1))) return bail(rc);
    const int maxblk = std::max({S.Q.nblk, S.A.nblk, S.AT.nblk, S.R.nblk, VEC_GRID_MAX});   // partials slots
    if ((rc = dalloc(h, &S.partials, (size_t)maxblk * 8 * 2))) return bail(rc);
    S.partials2 = S.partials + (size_t)maxblk * 8;
    if (S.qdiag && S.A.nlr > 0 && prox_diag_deferrable(S))
        if ((rc = dalloc(h, &S.ylr, (size_t)2 * S.A.nlr))) return bail(rc);
    if (hipMemsetAsync(S.ctrl, 0, sizeof(Ctrl), h->own) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipMemset failed"));

    // scalars of the problem
    qp_params d = qp_params_default();
    if ((rc = power_norm(h, S.A, S.AT, d.power_tol, d.power_max_iter, &h->norm_A))) return bail(rc);
    if (h->qkind == 2) {
        if ((rc = power_norm(h, S.Q, S.Q, d.power_tol, d.power_max_iter, &h->norm_Q_raw, true))) return bail(rc);
        h->norm_Q = d.norm_safety * h->norm_Q_raw;
    } else {
        h->norm_Q = 0.0;
        for (int64_t i = 0; i < n; ++i) h->norm_Q = std::max(h->norm_Q, std::fabs(qd[i]));
    }
    double nb = 0.0, nc = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        const double bt = std::isfinite(lc[i]) ? lc[i] : (std::isfinite(uc[i]) ? uc[i] : 0.0);
        nb += bt * bt;
    }
    for (int64_t i = 0; i < n; ++i) nc += c[i] * c[i];
    nb = std::sqrt(nb);
    nc = std::sqrt(nc);
    h->omega0 = (nc > 1e-10 && nb > 1e-10) ? nc / nb : 1.0;
    h->c_max = 0.0;
    for (int64_t i = 0; i < n; ++i) h->c_max = std::max(h->c_max, std::fabs(c[i]));
    double bl = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        if (std::isfinite(lc[i])) bl = std::max(bl, std::fabs(lc[i]));
        if (std::isfinite(uc[i])) bl = std::max(bl, std::fabs(uc[i]));
    }
    h->bscale_p = 1.0 + bl;
    h->gamma_q = 1.0;
    {
        // row sums of |Q|; for a factored Q the bound |P| + |R|'|R| 1
        std::vector<double> rs(n, 0.0);
        if (Qp)
            for (int64_t i = 0; i < n; ++i)
                for (int64_t e = Qp[i]; e < Qp[i + 1]; ++e) rs[i] += std::fabs(Qv[e]);
        if (k > 0) {
            std::vector<double> r1(k, 0.0);
            for (int64_t r = 0; r < k; ++r)
                for (int64_t e = Rp[r]; e < Rp[r + 1]; ++e) r1[r] += std::fabs(Rv[e]);
            for (int64_t i = 0; i < n; ++i)
                for (int64_t e = rtp[i]; e < rtp[i + 1]; ++e) rs[i] += std::fabs(rtv[e]) * r1[rtj[e]];
        }
        for (int64_t i = 0; i < n; ++i) h->gamma_q = std::max(h->gamma_q, rs[i]);
    }
    h->has_unbounded_x = 0;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(lvv[i]) || !std::isfinite(uvv[i])) h->has_unbounded_x = 1;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(QP_ERR_DEVICE, "setup failed"));
    h->setup_seconds = now_s() - t0;
    *out = h;
    g_err.clear();
    return 0;
}

// ---- timing of kernel families ----------------------------------------------

struct Timed {
    qp_handle* h;
    int fam;
    EventPair* ev = nullptr;
    Timed(qp_handle* hh, int f) : h(hh), fam(f)
    {
        const int64_t k = h->fam_launches[fam]++;
        if (h->timing > 0 && fam != QP_FAM_CHECK && k % h->timing == 0 &&
            h->ev_used < h->ev_pool.size()) {
            ev = &h->ev_pool[h->ev_used++];
            ev->fam = fam;
            h->S.tev = ev->ev;
        }
    }
    ~Timed() { h->S.tev = nullptr; }
};

void setup_ctrl(qp_handle* h, const qp_params& p, Ctrl& c)
{
    std::memset(&c, 0, sizeof(c));
    c.omega0 = h->omega0;
    c.omega = h->omega0;
    c.norm_A = h->norm_A;
    c.eta = h->norm_A * p.norm_safety > 1e-12 ? p.eta_scale / (p.norm_safety * h->norm_A) : 1.0;
    c.tau = c.eta / c.omega;
    c.sigma = c.eta * c.omega;
    c.inv_tau = 1.0 / c.tau;
    c.norm_Q = h->norm_Q;
    c.eps = INFINITY;
    c.gamma_inner = p.gamma_inner;
    c.eps_min = p.eps_min;
    c.eps_fixed = p.eps_inner_fixed;
    c.abar_scale = p.mprgp_abar_scale;
    c.abar = p.mprgp_abar_scale / (c.norm_Q + c.inv_tau);
    c.mprgp_gamma = p.mprgp_gamma;
    c.max_inner = p.max_inner;
    c.max_iter = p.max_iter;
    c.theta = p.theta;
    c.use_halpern = p.use_halpern;
    c.has_unbounded_x = h->has_unbounded_x;
    c.kp = p.kp; c.ki = p.ki; c.kd = p.kd;
    c.rs_suff = p.restart_sufficient;
    c.rs_nec = p.restart_necessary;
    c.rs_art = p.restart_artificial;
    c.tol = p.tol;
    c.eps_inf = p.eps_inf;
    c.c_max = h->c_max;
    c.bscale_p = h->bscale_p;
    c.gamma_q = h->gamma_q;
}

// Runs one inner solve (gradient at the warm start, then steps until the
// device posts "done").  The host keeps `lag` steps queued beyond the last
// status it has seen, so the GPU never waits for the host.
// `exact`: form rhs (already done by the caller) and the gradient with a
// product with Q; otherwise update both from the previous subproblem.
// K inner steps (direction, H p, update) as one graph: the steps take no
// per-step argument, so the same graph serves every subproblem of the handle
int ensure_inner_graph(qp_handle* h, int K)
{
    DevState& S = h->S;
    if (h->graph_exec && h->graph_steps == K && h->graph_mixed == S.mixed) return 0;
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    hipStream_t cs = h->own;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int k = 0; k < K && err == hipSuccess; ++k) {
        err = launch_dir(S, cs);
        if (err == hipSuccess) err = launch_hp(S, cs);
        if (err == hipSuccess) err = launch_update(S, cs);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(QP_ERR_DEVICE, std::string("graph capture failed: ") +
                                       hipGetErrorString(err != hipSuccess ? err : e2));
    }
    h->graph = g;
    HIPCHK(hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
    h->graph_steps = K;
    h->graph_mixed = S.mixed;
    return 0;
}

int inner_solve(qp_handle* h, long long& gseq, int lag, bool exact, int K, bool pre_xbar = false)
{
    DevState& S = h->S;
    hipStream_t s = h->stream;
    const long long base = gseq;
    if (exact) {
        Timed t(h, QP_FAM_GINIT);
        HIPCHK(launch_ginit(S, base, s));
    } else {
        Timed t(h, QP_FAM_RHS);
        HIPCHK(launch_rhs_grad(S, base, pre_xbar, s));
    }
    volatile unsigned long long* word = h->hstat;
    long long issued = 0;
    const int batch = K > 0 ? K : 1;   // inner steps per launch (graph or eager)
    for (;;) {
        const long long target = issued - (long long)lag * batch;
        if (target >= 0) {
            long long spins = 0;
            for (;;) {
                const unsigned long long w = *word;
                const long long sq = (long long)(w >> 1);
                if (sq >= base + target || (sq >= base && (w & 1ull))) break;
                if ((++spins & 0x3ff) == 0) {
                    const hipError_t q = hipStreamQuery(s);
                    if (q == hipSuccess) {
                        const unsigned long long w2 = *word;
                        const long long s2 = (long long)(w2 >> 1);
                        if (s2 >= base + target || (s2 >= base && (w2 & 1ull))) break;
                        return fail(QP_ERR_DEVICE, "inner solver posted no status (internal error)");
                    }
                    if (q != hipErrorNotReady)
                        return fail(QP_ERR_DEVICE, std::string("stream error: ") + hipGetErrorString(q));
                }
            }
        }
        const unsigned long long w = *word;
        if ((long long)(w >> 1) >= base && (w & 1ull)) break;
        if (K > 0) {
            HIPCHK(hipGraphLaunch(h->graph_exec, s));
            issued += K;
            h->fam_launches[QP_FAM_DIR] += K;
            h->fam_launches[QP_FAM_SPMV_HP] += K;
            h->fam_launches[QP_FAM_UPDATE] += K;
            continue;
        }
        ++issued;
        {
            Timed t(h, QP_FAM_DIR);
            HIPCHK(launch_dir(S, s));
        }
        {
            Timed t(h, QP_FAM_SPMV_HP);
            HIPCHK(launch_hp(S, s));
        }
        {
            Timed t(h, QP_FAM_UPDATE);
            HIPCHK(launch_update(S, s));
        }
    }
    gseq = base + issued + 1;
    return 0;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

qp_params qp_params_default(void)
{
    qp_params p;
    std::memset(&p, 0, sizeof(p));
    p.tol = 1e-6;
    p.max_iter = 100000;
    p.check_every = 64;
    p.max_inner = 500;
    p.use_halpern = 1;
    p.inner_lag = 1;
    p.theta = 1.0;
    p.kp = 0.99;
    p.ki = 0.01;
    p.kd = 0.0;
    p.gamma_inner = 5e-4;
    p.eps_min = 1e-9;
    p.eps_inner_fixed = 0.0;
    p.restart_sufficient = 0.2;
    p.restart_necessary = 0.8;
    p.restart_artificial = 0.36;
    p.eps_inf = 1e-8;
    p.eta_scale = 0.998;
    p.norm_safety = 1.01;
    p.power_tol = 1e-7;
    p.power_max_iter = 1000;
    p.mprgp_gamma = 1.0;
    p.mprgp_abar_scale = 1.9;
    p.timing = 0;
    p.precision = QP_PRECISION_FP64;
    p.graph_steps = 0;
    p.reserved = 0;
    return p;
}

const char* qp_last_error(void) { return g_err.c_str(); }

int qp_create(int64_t n, int64_t m, const int64_t* Q_rowptr, const int32_t* Q_col,
              const double* Q_val, const int64_t* A_rowptr, const int32_t* A_col,
              const double* A_val, const double* c, const double* b, const char* sense,
              const double* lb, const double* ub, qp_handle** out)
{
    if (!out) return fail(QP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= INT32_MAX || m < 0 || m >= INT32_MAX)
        return fail(QP_ERR_INVALID_ARG, "need 1 <= n < 2^31 and 0 <= m < 2^31");
    if (m > 0 && (!b || !sense)) return fail(QP_ERR_INVALID_ARG, "b or sense is NULL");
    int rc = check_vec("b", m, b, false);
    if (m > 0 && rc) return rc;
    std::vector<double> lc(m), uc(m);
    for (int64_t i = 0; i < m; ++i) {
        switch (sense[i]) {
        case 'E': lc[i] = b[i]; uc[i] = b[i]; break;
        case 'G': lc[i] = b[i]; uc[i] = INFINITY; break;
        case 'L': lc[i] = -INFINITY; uc[i] = b[i]; break;
        default: return fail(QP_ERR_INVALID_ARG, "sense: unknown character at row " + std::to_string(i));
        }
    }
    return create_impl(n, m, Q_rowptr, Q_col, Q_val, A_rowptr, A_col, A_val, c, lc.data(),
                       uc.data(), lb, ub, out);
}

int qp_create_ranged(int64_t n, int64_t m, const int64_t* Q_rowptr, const int32_t* Q_col,
                     const double* Q_val, const int64_t* A_rowptr, const int32_t* A_col,
                     const double* A_val, const double* c, const double* lc, const double* uc,
                     const double* lb, const double* ub, qp_handle** out)
{
    if (!out) return fail(QP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= INT32_MAX || m < 0 || m >= INT32_MAX)
        return fail(QP_ERR_INVALID_ARG, "need 1 <= n < 2^31 and 0 <= m < 2^31");
    if (m > 0 && (!lc || !uc)) return fail(QP_ERR_INVALID_ARG, "lc or uc is NULL");
    std::vector<double> l(m), u(m);
    for (int64_t i = 0; i < m; ++i) { l[i] = lc[i]; u[i] = uc[i]; }
    int rc = check_bounds("lc/uc", m, l.data(), u.data());
    if (rc) return rc;
    return create_impl(n, m, Q_rowptr, Q_col, Q_val, A_rowptr, A_col, A_val, c, l.data(),
                       u.data(), lb, ub, out);
}

int qp_create_factored(int64_t n, int64_t m, const int64_t* P_rowptr, const int32_t* P_col,
                       const double* P_val, int64_t k, const int64_t* R_rowptr, const int32_t* R_col,
                       const double* R_val, const int64_t* A_rowptr, const int32_t* A_col,
                       const double* A_val, const double* c, const double* b, const char* sense,
                       const double* lb, const double* ub, qp_handle** out)
{
    if (!out) return fail(QP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= INT32_MAX || m < 0 || m >= INT32_MAX)
        return fail(QP_ERR_INVALID_ARG, "need 1 <= n < 2^31 and 0 <= m < 2^31");
    if (k < 1) return fail(QP_ERR_INVALID_ARG, "need k >= 1 (use qp_create without factors)");
    if (m > 0 && (!b || !sense)) return fail(QP_ERR_INVALID_ARG, "b or sense is NULL");
    int rc = check_vec("b", m, b, false);
    if (m > 0 && rc) return rc;
    std::vector<double> lc(m), uc(m);
    for (int64_t i = 0; i < m; ++i) {
        switch (sense[i]) {
        case 'E': lc[i] = b[i]; uc[i] = b[i]; break;
        case 'G': lc[i] = b[i]; uc[i] = INFINITY; break;
        case 'L': lc[i] = -INFINITY; uc[i] = b[i]; break;
        default: return fail(QP_ERR_INVALID_ARG, "sense: unknown character at row " + std::to_string(i));
        }
    }
    return create_impl(n, m, P_rowptr, P_col, P_val, A_rowptr, A_col, A_val, c, lc.data(), uc.data(), lb, ub,
                       out, k, R_rowptr, R_col, R_val);
}

int qp_set_stream(qp_handle* h, void* stream)
{
    if (!h) return fail(QP_ERR_INVALID_ARG, "handle is NULL");
    h->stream = stream ? static_cast<hipStream_t>(stream) : h->own;
    return 0;
}

void qp_destroy(qp_handle* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->own) {
        for (void* p : h->dev_allocs) (void)hipFreeAsync(p, h->own);
        (void)hipStreamSynchronize(h->own);
    }
    for (EventPair& e : h->ev_pool) {
        (void)hipEventDestroy(e.ev[0]);
        (void)hipEventDestroy(e.ev[1]);
    }
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->hstat) (void)hipHostFree(h->hstat);
    if (h->own) (void)hipStreamDestroy(h->own);
    delete h;
}

int qp_solve(qp_handle* h, double tol, int64_t max_iter)
{
    qp_params p = qp_params_default();
    p.tol = tol;
    p.max_iter = max_iter;
    return qp_solve_ex(h, &p);
}

int qp_solve_ex(qp_handle* h, const qp_params* params)
{
    if (!h) return fail(QP_ERR_INVALID_ARG, "handle is NULL");
    const qp_params p = params ? *params : qp_params_default();
    if (!(p.tol > 0.0) || p.max_iter < 0 || p.check_every < 1 || p.max_inner < 0 || p.inner_lag < 0 ||
        (p.precision != QP_PRECISION_FP64 && p.precision != QP_PRECISION_MIXED) || p.graph_steps < 0 ||
        p.graph_steps > 64)
        return fail(QP_ERR_INVALID_ARG, "invalid parameters");
    DevState& S = h->S;
    hipStream_t s = h->stream;
    const double t0 = now_s();
    if (int rc = set_precision(h, p.precision)) return rc;
    // inner steps per graph launch (eager launches when timing kernel families)
    const int K = (p.timing > 0 || S.qdiag) ? 0 : p.graph_steps;
    if (K > 0)
        if (int rc = ensure_inner_graph(h, K)) return rc;

    h->timing = p.timing;
    std::fill(h->fam_launches, h->fam_launches + QP_NFAM, 0);
    h->ev_used = 0;
    if (p.timing > 0 && h->ev_pool.empty()) {
        h->ev_pool.resize(4096);
        for (EventPair& e : h->ev_pool) {
            HIPCHK(hipEventCreate(&e.ev[0]));
            HIPCHK(hipEventCreate(&e.ev[1]));
        }
    }

    Ctrl c;
    setup_ctrl(h, p, c);
    HIPCHK(hipMemcpyAsync(S.ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    HIPCHK(launch_init_start(S, s));
    HIPCHK(launch_ref_zero(S, s));
    HIPCHK(hipStreamSynchronize(s));
    h->hstat[0] = 0;
    h->hstat[1] = 0;

    long long gseq = 1;
    int64_t k = 0;
    long long nchecks = 0;
    // the round's step count t, tracked here for the closed-form path (the
    // device resets it at a restart, which only a check decides and posts)
    long long t_round = 0;
    bool xbar_pending = false;   // the last x_bar kernel's finishing work is still to run
    // closed-form path: the dual step of iteration lr_k (round step lr_t) left
    // its long rows to the next primal kernel (-1: none)
    long long lr_k = -1, lr_t = -1;
    int status = QP_NOT_SOLVED;
    for (;;) {
        if (k > 0 || p.max_iter == 0) {
            if (k % p.check_every == 0 || k >= p.max_iter) {
                {
                    Timed t(h, QP_FAM_CHECK);
                    HIPCHK(launch_check(S, S.xt, S.yt, 1, h->has_unbounded_x, s));
                    HIPCHK(launch_restart_copy(S, s));
                    HIPCHK(launch_ref_update(S, s));
                }
                // the decision is in the pinned check word once the stream
                // has drained: no device-to-host copies (each a blit launch
                // and a second sync; together about 110 us per check).
                // Spinning on the word instead of the sync measured no
                // faster alone and slower for a server's concurrent solves.
                HIPCHK(hipStreamSynchronize(s));
                const unsigned long long word = *(volatile unsigned long long*)h->hcheck;
                if ((long long)(word >> 2) != ++nchecks)
                    return fail(QP_ERR_DEVICE, "check posted no decision (internal error)");
                if (word & 1ull) {
                    int st = 0;
                    HIPCHK(hipStreamSynchronize(s));
                    HIPCHK(copy_wait(&st, &S.ctrl->status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
                    status = st;
                    break;
                }
                if (word & 2ull) t_round = 0;
            }
        }
        if (k >= p.max_iter) {
            status = QP_ITERATION_LIMIT;
            break;
        }
        const int next_check = ((k + 1) % p.check_every == 0) || (k + 1 >= p.max_iter);
        // the movement norms and certificate pieces are read only at the
        // round's first step (the restart test's reference) and before a
        // check: the other iterations skip the dual step's reductions and
        // finishing step (a non-diagonal Q's x_bar finishing work, which
        // updates the inner tolerance, then rides with the next iteration's
        // right-hand side instead)
        const bool reduce = next_check || t_round == 0;
        if (S.qdiag) {
            Timed t(h, QP_FAM_RHS);
            HIPCHK(launch_prox_diag(S, next_check, t_round, reduce, lr_k, lr_t, s));
            lr_k = lr_t = -1;
        } else {
            // the gradient is formed with a product with Q at the first
            // iteration and after every check (bounds the drift of the
            // recurrence to check_every iterations); otherwise it is updated
            const bool exact = (k % p.check_every == 0);
            if (exact) {
                Timed t(h, QP_FAM_RHS);
                HIPCHK(launch_rhs(S, s));
            }
            int rc = inner_solve(h, gseq, p.inner_lag, exact, K, xbar_pending);
            if (rc) return rc;
            Timed t(h, QP_FAM_HALPX);
            HIPCHK(launch_xbar(S, next_check, t_round, s));
        }
        {
            Timed t(h, QP_FAM_DUAL);
            const int pre = S.qdiag ? (prox_diag_deferrable(S) ? PRE_PROX : PRE_NONE) : PRE_XBAR;
            // a step whose reductions nothing reads leaves its long rows to
            // the next primal kernel (never before a check: that iteration reduces)
            const bool leave_long = S.ylr != nullptr && !reduce;
            HIPCHK(launch_dual(S, next_check, pre, t_round, k, reduce, leave_long, s));
            if (leave_long) {
                lr_k = k;
                lr_t = t_round;
            }
            xbar_pending = !S.qdiag && !reduce;
        }
        ++k;
        ++t_round;
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t1 = now_s();

    Ctrl r;
    HIPCHK(copy_wait(&r, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    qp_info& I = h->info;
    std::memset(&I, 0, sizeof(I));
    I.status = status;
    I.precision = p.precision;
    I.iterations = r.k;
    I.inner_iterations = r.inner_total;
    I.restarts = r.restarts;
    I.checks = r.checks;
    I.r_primal = r.r_primal;
    I.r_dual = r.r_dual;
    I.r_gap = r.r_gap;
    I.primal_obj = r.pobj;
    I.dual_obj = r.dobj;
    I.natural_residual = r.natural;
    I.omega = r.omega;
    I.eta = r.eta;
    I.norm_A = h->norm_A;
    I.norm_Q = h->norm_Q;
    I.eps_inner = r.eps;
    I.solve_seconds = t1 - t0;
    I.setup_seconds = h->setup_seconds;
    for (int f = 0; f < QP_NFAM; ++f) I.fam_launches[f] = h->fam_launches[f];
    I.spmv_hp_active = r.hp_active;
    for (size_t i = 0; i < h->ev_used; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->ev_pool[i].ev[0], h->ev_pool[i].ev[1]) == hipSuccess) {
            I.fam_ms[h->ev_pool[i].fam] += ms;
            I.fam_timed[h->ev_pool[i].fam] += 1;
        }
    }
    h->status = status;
    h->solved = 1;
    g_err.clear();
    return status;
}

int qp_result(const qp_handle* h, double* x, double* y, qp_info* info)
{
    if (!h) return fail(QP_ERR_INVALID_ARG, "handle is NULL");
    if (!h->solved) return fail(QP_ERR_STATE, "no solve has run on this handle");
    const DevState& S = h->S;
    Ctrl r;
    HIPCHK(copy_wait(&r, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    if (x) {
        if (h->status == QP_DUAL_INFEASIBLE) {
            HIPCHK(copy_wait(x, S.dx, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
            for (int64_t i = 0; i < h->n; ++i) x[i] /= r.d_max;
        } else {
            HIPCHK(copy_wait(x, S.xt, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
        }
    }
    if (y && h->m > 0) {
        if (h->status == QP_PRIMAL_INFEASIBLE) {
            HIPCHK(copy_wait(y, S.ytil, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->stream));
            for (int64_t i = 0; i < h->m; ++i) y[i] /= r.ytil_max;
        } else {
            HIPCHK(copy_wait(y, S.yt, sizeof(double) * h->m, hipMemcpyDeviceToHost, h->stream));
        }
    }
    if (info) *info = h->info;
    return h->status;
}

int qp_apply(qp_handle* h, int op, const double* x, double* y)
{
    if (!h || !x || !y) return fail(QP_ERR_INVALID_ARG, "NULL argument");
    const CsrDev* M = op == QP_OP_Q ? &h->S.Q : op == QP_OP_A ? &h->S.A : op == QP_OP_AT ? &h->S.AT : nullptr;
    if (!M) return fail(QP_ERR_INVALID_ARG, "unknown operator");
    if (op == QP_OP_Q && h->S.k > 0) {
        // [P | R'] on [x; R x]
        HIPCHK(hipMemcpyAsync(h->S.v1, x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(launch_tail(h->S, h->S.v1, h->S.v1 + h->n, false, h->stream));
        x = h->S.v1;
    }
    HIPCHK(launch_spmv_plain(h->S, *M, x, y, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

int qp_dot(qp_handle* h, int64_t len, const double* a, const double* b, double* out)
{
    if (!h || !out || len < 0 || len >= INT32_MAX || (len > 0 && (!a || !b)))
        return fail(QP_ERR_INVALID_ARG, "bad argument");
    HIPCHK(launch_dot(h->S, a, b, (int)len, h->stream));
    HIPCHK(hipMemcpyAsync(&h->hcheck[1], &h->S.ctrl->pw_norm, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::memcpy(out, &h->hcheck[1], sizeof(double));
    return 0;
}

int qp_subproblem(qp_handle* h, double tau, const double* rhs, double* x, double eps,
                  int64_t max_inner, int64_t* iters, double* res)
{
    if (!h || !rhs || !x || !(tau > 0.0) || max_inner < 0 || !(eps >= 0.0))
        return fail(QP_ERR_INVALID_ARG, "bad argument");
    DevState& S = h->S;
    hipStream_t s = h->stream;
    qp_params p = qp_params_default();
    if (int rc = set_precision(h, QP_PRECISION_FP64)) return rc;
    Ctrl c;
    setup_ctrl(h, p, c);
    c.tau = tau;
    c.inv_tau = 1.0 / tau;
    c.abar = p.mprgp_abar_scale / (c.norm_Q + c.inv_tau);
    c.eps = eps;
    c.eps_fixed = eps > 0.0 ? eps : 1e-300;
    c.max_inner = max_inner;
    HIPCHK(hipMemcpyAsync(S.ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(S.rhs, rhs, sizeof(double) * h->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(S.xt, x, sizeof(double) * h->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_clip(S, S.xt, s));
    HIPCHK(hipStreamSynchronize(s));
    h->hstat[0] = 0;
    long long gseq = 1;
    int rc = inner_solve(h, gseq, 2, true, 0);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(x, S.xt, sizeof(double) * h->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    Ctrl r;
    HIPCHK(copy_wait(&r, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    if (iters) *iters = r.inner_it;
    if (res) *res = r.res;
    return 0;
}

int qp_kkt(qp_handle* h, const double* x, const double* y, double* out)
{
    if (!h || !x || (!y && h->m > 0) || !out) return fail(QP_ERR_INVALID_ARG, "NULL argument");
    DevState& S = h->S;
    hipStream_t s = h->stream;
    Ctrl c;
    setup_ctrl(h, qp_params_default(), c);
    HIPCHK(hipMemcpyAsync(S.ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    HIPCHK(launch_check(S, x, y ? y : S.y, 0, 0, s));
    HIPCHK(hipStreamSynchronize(s));
    Ctrl r;
    HIPCHK(copy_wait(&r, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    out[0] = r.r_primal; out[1] = r.r_dual; out[2] = r.r_gap;
    out[3] = r.pobj; out[4] = r.dobj; out[5] = r.natural; out[6] = r.pviol;
    return 0;
}

// ===========================================================================
// batched solve
// ===========================================================================

}  // extern "C"

struct qp_batch {
    int64_t count = 0, n = 0, m = 0;
    std::vector<int64_t> voff, roff;
    BatchDev B;
    hipStream_t stream = nullptr;
    bool own_stream = true;        // false: a stream lent by the caller (not destroyed)
    hipEvent_t done = nullptr;
    double t_launch = 0.0;
    int64_t nnz_a = 0, nnz_q = 0;
    float *a32 = nullptr, *t32 = nullptr, *q32 = nullptr;   // made at the first mixed solve
    std::vector<void*> allocs;
    Arena* arena = nullptr;        // set: device buffers come from the caller's region (none freed)
    std::vector<BatchOut> out;
    std::vector<double> norm_A;
    // launch schedule: shape (index into the compiled table) and queue order
    // (0 index order, 1 largest instance first; dorder holds that permutation)
    int shape = pdhcg::BATCH_SHAPE_DEFAULT, order = 1;
    const int* dorder = nullptr;
    int solved = 0;
    double setup_seconds = 0.0, solve_seconds = 0.0;
};

namespace {

template <class T>
int balloc(qp_batch* bt, T** p, size_t count)
{
    void* q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (Arena* a = bt->arena) {
        const size_t at = (a->used + 255) & ~(size_t)255;
        if (at > a->cap || bytes > a->cap - at)
            return fail(QP_ERR_INVALID_ARG, "the batch needs more device memory than the static workspace's " +
                                                std::to_string(a->cap) + " bytes");
        a->used = at + bytes;
        *p = reinterpret_cast<T*>(a->base + at);
        return 0;
    }
    hipError_t e = hipMallocAsync(&q, bytes, bt->stream);
    if (e != hipSuccess) return fail(QP_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    bt->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return 0;
}

template <class T>
int bupload(qp_batch* bt, const T** p, const T* src, size_t count)
{
    T* q = nullptr;
    int rc = balloc(bt, &q, count);
    if (rc) return rc;
    if (count) HIPCHK(copy_wait(q, src, count * sizeof(T), hipMemcpyHostToDevice, bt->stream));
    *p = q;
    return 0;
}

}  // namespace

extern "C" {

void qp_batch_destroy(qp_batch* bt)
{
    if (!bt) return;
    if (bt->stream || bt->arena) {
        (void)hipStreamSynchronize(bt->stream);
        for (void* p : bt->allocs) (void)hipFreeAsync(p, bt->stream);
        (void)hipStreamSynchronize(bt->stream);
    }
    if (bt->done) (void)hipEventDestroy(bt->done);
    if (bt->stream && bt->own_stream) (void)hipStreamDestroy(bt->stream);
    delete bt;
}

int qp_batch_create(int64_t count, const int64_t* var_off, const int64_t* row_off,
                    const int64_t* Qp, const int32_t* Qj, const double* Qv,
                    const int64_t* Ap, const int32_t* Aj, const double* Av,
                    const double* c, const double* b, const char* sense,
                    const double* lb, const double* ub, qp_batch** out)
{
    return pdhcg::batch_create(nullptr, count, var_off, row_off, Qp, Qj, Qv, Ap, Aj, Av, c, b, sense, lb,
                               ub, out);
}

}  // extern "C"

namespace pdhcg {

int batch_create(hipStream_t lane, int64_t count, const int64_t* var_off, const int64_t* row_off,
                 const int64_t* Qp, const int32_t* Qj, const double* Qv,
                 const int64_t* Ap, const int32_t* Aj, const double* Av,
                 const double* c, const double* b, const char* sense,
                 const double* lb, const double* ub, qp_batch** out, Arena* arena)
{
    const double t0 = now_s();
    if (!out) return fail(QP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || count >= INT32_MAX || !var_off || !row_off)
        return fail(QP_ERR_INVALID_ARG, "need count >= 1 and instance offsets");
    if (var_off[0] != 0 || row_off[0] != 0) return fail(QP_ERR_INVALID_ARG, "offsets must start at 0");
    for (int64_t i = 0; i < count; ++i) {
        if (var_off[i + 1] <= var_off[i]) return fail(QP_ERR_INVALID_ARG, "every instance needs >= 1 variable");
        if (row_off[i + 1] < row_off[i]) return fail(QP_ERR_INVALID_ARG, "row offsets decrease");
    }
    const int64_t n = var_off[count], m = row_off[count];
    if (n >= INT32_MAX || m >= INT32_MAX) return fail(QP_ERR_INVALID_ARG, "n and m must be below 2^31");
    int rc;
    std::vector<double> lvv(n), uvv(n), lcv(m), ucv(m);
    for (int64_t i = 0; i < n; ++i) {
        lvv[i] = lb ? lb[i] : -INFINITY;
        uvv[i] = ub ? ub[i] : INFINITY;
    }
    if ((rc = check_bounds("lb/ub", n, lvv.data(), uvv.data()))) return rc;
    if ((rc = check_vec("c", n, c, false))) return rc;
    if (m > 0) {
        if (!b || !sense) return fail(QP_ERR_INVALID_ARG, "b or sense is NULL");
        if ((rc = check_vec("b", m, b, false))) return rc;
    }
    for (int64_t i = 0; i < m; ++i) {
        switch (sense[i]) {
        case 'E': lcv[i] = b[i]; ucv[i] = b[i]; break;
        case 'G': lcv[i] = b[i]; ucv[i] = INFINITY; break;
        case 'L': lcv[i] = -INFINITY; ucv[i] = b[i]; break;
        default: return fail(QP_ERR_INVALID_ARG, "sense: unknown character at row " + std::to_string(i));
        }
    }
    std::vector<int64_t> a_empty(1, 0);
    if (!Ap) {
        if (m != 0) return fail(QP_ERR_INVALID_ARG, "A: row pointer is NULL");
        Ap = a_empty.data();
    }
    if ((rc = check_csr("A", m, n, Ap, Aj, Av))) return rc;
    std::vector<double> qd(n, 0.0);
    std::vector<int> qgen(count, 0);
    std::vector<int64_t> q_empty(n + 1, 0);
    if (Qp) {
        if ((rc = check_csr("Q", n, n, Qp, Qj, Qv))) return rc;
        if ((rc = check_symmetric(n, Qp, Qj, Qv))) return rc;
        for (int64_t b = 0; b < count; ++b)
            for (int64_t i = var_off[b]; i < var_off[b + 1]; ++i)
                for (int64_t k = Qp[i]; k < Qp[i + 1]; ++k) {
                    if (Qj[k] < var_off[b] || Qj[k] >= var_off[b + 1])
                        return fail(QP_ERR_INVALID_ARG, "Q is not block-diagonal at row " + std::to_string(i));
                    if (Qj[k] != i) qgen[b] = 1;
                    else qd[i] += Qv[k];
                }
    } else {
        Qp = q_empty.data();
    }
    for (int64_t i = 0; i < count; ++i)
        for (int64_t r = row_off[i]; r < row_off[i + 1]; ++r)
            for (int64_t k = Ap[r]; k < Ap[r + 1]; ++k)
                if (Aj[k] < var_off[i] || Aj[k] >= var_off[i + 1])
                    return fail(QP_ERR_INVALID_ARG, "A is not block-diagonal at row " + std::to_string(r));
    // the kernel sums each row with one thread; rows longer than
    // QP_BATCH_MAX_ROW nonzeros (of A, A' or Q) are not accepted
    {
        std::vector<int64_t> colcnt(n, 0);
        for (int64_t k = 0; k < Ap[m]; ++k) ++colcnt[Aj[k]];
        for (int64_t r = 0; r < m; ++r)
            if (Ap[r + 1] - Ap[r] > QP_BATCH_MAX_ROW)
                return fail(QP_ERR_INVALID_ARG, "row " + std::to_string(r) + " of A is longer than QP_BATCH_MAX_ROW");
        for (int64_t j = 0; j < n; ++j)
            if (colcnt[j] > QP_BATCH_MAX_ROW || Qp[j + 1] - Qp[j] > QP_BATCH_MAX_ROW)
                return fail(QP_ERR_INVALID_ARG,
                            "column " + std::to_string(j) + " of A or row of Q is longer than QP_BATCH_MAX_ROW");
    }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(QP_ERR_DEVICE, "no HIP device available");
    qp_batch* bt = new qp_batch();
    auto bail = [&](int code) { qp_batch_destroy(bt); return code; };
    bt->count = count;
    bt->n = n;
    bt->m = m;
    bt->voff.assign(var_off, var_off + count + 1);
    bt->roff.assign(row_off, row_off + count + 1);
    bt->arena = arena;
    if (lane || arena) {
        bt->stream = lane;
        bt->own_stream = false;
    } else if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess) {
        return bail(fail(QP_ERR_DEVICE, "hipStreamCreate failed"));
    }
    // without an event (arena mode) the batch waits on its stream instead
    if (!arena && hipEventCreateWithFlags(&bt->done, hipEventDisableTiming) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipEventCreate failed"));
    BatchDev& B = bt->B;
    B.count = (int)count;
    std::vector<int> vo32(count + 1), ro32(count + 1), arp32(m + 1);
    for (int64_t i = 0; i <= count; ++i) { vo32[i] = (int)var_off[i]; ro32[i] = (int)row_off[i]; }
    for (int64_t i = 0; i <= m; ++i) arp32[i] = (int)Ap[i];
    std::vector<int64_t> tp;
    std::vector<int32_t> tj;
    std::vector<double> tv;
    transpose(m, n, Ap, Aj, Av, tp, tj, tv);
    std::vector<int> trp32(n + 1), qrp32(n + 1);
    for (int64_t i = 0; i <= n; ++i) { trp32[i] = (int)tp[i]; qrp32[i] = (int)Qp[i]; }
    const int64_t nnz = Ap[m], qnnz = Qp[n];
    bt->nnz_a = nnz;
    bt->nnz_q = qnnz;
    if ((rc = bupload(bt, &B.qrp, qrp32.data(), qrp32.size())) || (rc = bupload(bt, &B.qcol, Qj, (size_t)qnnz)) ||
        (rc = bupload(bt, &B.qval, Qv, (size_t)qnnz)))
        return bail(rc);
    if ((rc = bupload(bt, &B.voff, vo32.data(), vo32.size())) || (rc = bupload(bt, &B.roff, ro32.data(), ro32.size())) ||
        (rc = bupload(bt, &B.arp, arp32.data(), arp32.size())) || (rc = bupload(bt, &B.acol, Aj, (size_t)nnz)) ||
        (rc = bupload(bt, &B.aval, Av, (size_t)nnz)) || (rc = bupload(bt, &B.trp, trp32.data(), trp32.size())) ||
        (rc = bupload(bt, &B.tcol, tj.data(), tj.size())) || (rc = bupload(bt, &B.tval, tv.data(), tv.size())) ||
        (rc = bupload(bt, &B.qd, qd.data(), (size_t)n)) || (rc = bupload(bt, &B.c, c, (size_t)n)) ||
        (rc = bupload(bt, &B.lc, lcv.data(), (size_t)m)) || (rc = bupload(bt, &B.uc, ucv.data(), (size_t)m)))
        return bail(rc);
    {
        // the box as one pair, byte classes or arrays (as for one problem)
        std::vector<unsigned char> cls;
        std::vector<double> tl, tu;
        const int mode = classify_bounds(lvv, uvv, cls, tl, tu);
        B.lv.mode = B.uv.mode = mode;
        if (mode == 1) {
            B.lv.k = tl[0];
            B.uv.k = tu[0];
        } else if (mode == 2) {
            if ((rc = bupload(bt, &B.lv.cls, cls.data(), cls.size())) ||
                (rc = bupload(bt, &B.lv.tab, tl.data(), tl.size())) || (rc = bupload(bt, &B.uv.tab, tu.data(), tu.size())))
                return bail(rc);
            B.uv.cls = B.lv.cls;
        } else {
            if ((rc = bupload(bt, &B.lv.a, lvv.data(), (size_t)n)) || (rc = bupload(bt, &B.uv.a, uvv.data(), (size_t)n)))
                return bail(rc);
        }
    }
    {
        // 16-bit column indices local to the instance when every instance
        // is small enough (the blocks were checked to be diagonal above)
        bool small = true;
        for (int64_t i = 0; i < count && small; ++i)
            small = var_off[i + 1] - var_off[i] <= 65536 && row_off[i + 1] - row_off[i] <= 65536;
        if (small) {
            std::vector<unsigned short> a16((size_t)nnz), t16(tj.size()), q16((size_t)qnnz);
            for (int64_t i = 0; i < count; ++i) {
                for (int64_t r = row_off[i]; r < row_off[i + 1]; ++r)
                    for (int64_t q = Ap[r]; q < Ap[r + 1]; ++q) a16[q] = (unsigned short)(Aj[q] - var_off[i]);
                for (int64_t v = var_off[i]; v < var_off[i + 1]; ++v) {
                    for (int64_t q = tp[v]; q < tp[v + 1]; ++q) t16[q] = (unsigned short)(tj[q] - row_off[i]);
                    for (int64_t q = Qp[v]; q < Qp[v + 1]; ++q) q16[q] = (unsigned short)(Qj[q] - var_off[i]);
                }
            }
            if ((rc = bupload(bt, &B.acol16, a16.data(), a16.size())) ||
                (rc = bupload(bt, &B.tcol16, t16.data(), t16.size())) ||
                (rc = bupload(bt, &B.qcol16, q16.data(), q16.size())))
                return bail(rc);
        }
    }
    double** nv[] = {&B.x, &B.xa, &B.xt, &B.xbar, &B.aty, &B.d, &B.rhs, &B.g, &B.p, &B.hp, &B.xref};
    for (double** p : nv)
        if ((rc = balloc(bt, p, (size_t)n))) return bail(rc);
    double** mv[] = {&B.y, &B.ya, &B.yt, &B.ytil, &B.yref, &B.axref};
    for (double** p : mv)
        if ((rc = balloc(bt, p, (size_t)m))) return bail(rc);
    if ((rc = balloc(bt, &B.queue, 1)) || (rc = balloc(bt, &B.out, (size_t)count))) return bail(rc);
    {
        // largest instance first (nonzeros of A and Q plus n + m), ties in
        // index order: a longest-processing-time-first queue, so the launch
        // does not end on one large instance started last
        std::vector<int64_t> work(count);
        for (int64_t i = 0; i < count; ++i)
            work[i] = (Ap[row_off[i + 1]] - Ap[row_off[i]]) + (Qp[var_off[i + 1]] - Qp[var_off[i]]) +
                      (var_off[i + 1] - var_off[i]) + (row_off[i + 1] - row_off[i]);
        std::vector<int> perm(count);
        for (int64_t i = 0; i < count; ++i) perm[i] = (int)i;
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b_) { return work[a] > work[b_]; });
        if ((rc = bupload(bt, &bt->dorder, perm.data(), perm.size()))) return bail(rc);
        B.order = bt->dorder;
    }

    // per-instance scalars: ||A_i||_2 on the device, the rest here
    double* dnorm = nullptr;
    if ((rc = balloc(bt, &dnorm, (size_t)count))) return bail(rc);
    const qp_params dp = qp_params_default();
    if (hipMemsetAsync(B.queue, 0, sizeof(int), bt->stream) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipMemsetAsync failed"));
    if (launch_batch_norm(B, BATCH_SHAPE_NORM, B.roff, B.voff, B.arp, B.acol, B.aval, B.trp, B.tcol, B.tval, nullptr,
                          dp.power_tol, dp.power_max_iter, B.x, B.y, B.xt, dnorm, bt->stream) != hipSuccess ||
        hipStreamSynchronize(bt->stream) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "norm kernel failed"));
    bt->norm_A.resize(count);
    if (copy_wait(bt->norm_A.data(), dnorm, sizeof(double) * count, hipMemcpyDeviceToHost, bt->stream) != hipSuccess)
        return bail(fail(QP_ERR_DEVICE, "hipMemcpy failed"));
    // ||Q_b||_2 for the instances with a non-diagonal Q (Q symmetric: Q' = Q)
    std::vector<double> normq_raw(count, 0.0);
    {
        const int* dsel = nullptr;
        if ((rc = bupload(bt, &dsel, qgen.data(), (size_t)count))) return bail(rc);
        B.qgen = dsel;
        if (hipMemsetAsync(B.queue, 0, sizeof(int), bt->stream) != hipSuccess ||
            launch_batch_norm(B, BATCH_SHAPE_NORM, B.voff, B.voff, B.qrp, B.qcol, B.qval, B.qrp, B.qcol, B.qval, dsel,
                              dp.power_tol, dp.power_max_iter, B.x, B.xa, B.xt, dnorm, bt->stream) != hipSuccess ||
            hipStreamSynchronize(bt->stream) != hipSuccess ||
            copy_wait(normq_raw.data(), dnorm, sizeof(double) * count, hipMemcpyDeviceToHost, bt->stream) != hipSuccess)
            return bail(fail(QP_ERR_DEVICE, "norm kernel failed"));
    }
    std::vector<double> eta(count), om0(count), cmax(count), bsc(count), gq(count), nq(count);
    std::vector<int> unb(count, 0);
    for (int64_t i = 0; i < count; ++i) {
        const double na = bt->norm_A[i];
        eta[i] = na * dp.norm_safety > 1e-12 ? dp.eta_scale / (dp.norm_safety * na) : 1.0;
        double nb = 0.0, nc = 0.0, cm = 0.0, bl = 0.0, g = 1.0;
        for (int64_t r = row_off[i]; r < row_off[i + 1]; ++r) {
            const double bt_ = std::isfinite(lcv[r]) ? lcv[r] : (std::isfinite(ucv[r]) ? ucv[r] : 0.0);
            nb += bt_ * bt_;
            if (std::isfinite(lcv[r])) bl = std::max(bl, std::fabs(lcv[r]));
            if (std::isfinite(ucv[r])) bl = std::max(bl, std::fabs(ucv[r]));
        }
        double qmax = 0.0;
        for (int64_t v = var_off[i]; v < var_off[i + 1]; ++v) {
            nc += c[v] * c[v];
            cm = std::max(cm, std::fabs(c[v]));
            double rs = 0.0;
            for (int64_t k = Qp[v]; k < Qp[v + 1]; ++k) rs += std::fabs(Qv[k]);
            g = std::max(g, rs);
            qmax = std::max(qmax, std::fabs(qd[v]));
            if (!std::isfinite(lvv[v]) || !std::isfinite(uvv[v])) unb[i] = 1;
        }
        nq[i] = qgen[i] ? dp.norm_safety * normq_raw[i] : qmax;
        nb = std::sqrt(nb);
        nc = std::sqrt(nc);
        om0[i] = (nc > 1e-10 && nb > 1e-10) ? nc / nb : 1.0;
        cmax[i] = cm;
        bsc[i] = 1.0 + bl;
        gq[i] = g;
    }
    if ((rc = bupload(bt, &B.eta, eta.data(), (size_t)count)) || (rc = bupload(bt, &B.omega0, om0.data(), (size_t)count)) ||
        (rc = bupload(bt, &B.cmax, cmax.data(), (size_t)count)) || (rc = bupload(bt, &B.bscale, bsc.data(), (size_t)count)) ||
        (rc = bupload(bt, &B.gammaq, gq.data(), (size_t)count)) || (rc = bupload(bt, &B.unb, unb.data(), (size_t)count)) ||
        (rc = bupload(bt, &B.normq, nq.data(), (size_t)count)))
        return bail(rc);
    bt->setup_seconds = now_s() - t0;
    *out = bt;
    g_err.clear();
    return 0;
}

int batch_launch(qp_batch* bt, const qp_params* params)
{
    if (!bt) return fail(QP_ERR_INVALID_ARG, "batch is NULL");
    const qp_params p = params ? *params : qp_params_default();
    if (!(p.tol > 0.0) || p.max_iter < 0 || p.check_every < 1 ||
        (p.precision != QP_PRECISION_FP64 && p.precision != QP_PRECISION_MIXED))
        return fail(QP_ERR_INVALID_ARG, "invalid parameters");
    if (p.precision == QP_PRECISION_MIXED) {
        if (!bt->a32) {
            int rc;
            if ((rc = balloc(bt, &bt->a32, (size_t)bt->nnz_a)) || (rc = balloc(bt, &bt->t32, (size_t)bt->nnz_a)) ||
                (rc = balloc(bt, &bt->q32, (size_t)bt->nnz_q)))
                return rc;
            HIPCHK(launch_to_f32(bt->B.aval, bt->a32, bt->nnz_a, bt->stream));
            HIPCHK(launch_to_f32(bt->B.tval, bt->t32, bt->nnz_a, bt->stream));
            HIPCHK(launch_to_f32(bt->B.qval, bt->q32, bt->nnz_q, bt->stream));
        }
        bt->B.aval32 = bt->a32; bt->B.tval32 = bt->t32; bt->B.qval32 = bt->q32;
    } else {
        bt->B.aval32 = bt->B.tval32 = bt->B.qval32 = nullptr;
    }
    BatchParams P{};
    P.tol = p.tol; P.eps_inf = p.eps_inf; P.theta = p.theta;
    P.kp = p.kp; P.ki = p.ki; P.kd = p.kd;
    P.rs_suff = p.restart_sufficient; P.rs_nec = p.restart_necessary; P.rs_art = p.restart_artificial;
    P.max_iter = p.max_iter; P.check_every = p.check_every; P.use_halpern = p.use_halpern;
    P.gamma_inner = p.gamma_inner; P.eps_min = p.eps_min; P.eps_fixed = p.eps_inner_fixed;
    P.mprgp_gamma = p.mprgp_gamma; P.abar_scale = p.mprgp_abar_scale; P.max_inner = p.max_inner;
    bt->t_launch = now_s();
    HIPCHK(hipMemsetAsync(bt->B.queue, 0, sizeof(int), bt->stream));
    bt->B.order = bt->order ? bt->dorder : nullptr;
    HIPCHK(launch_batch_solve(bt->B, P, bt->shape, bt->stream));
    if (bt->done) HIPCHK(hipEventRecord(bt->done, bt->stream));
    return 0;
}

// 1 when the launched solve has finished, 0 while it runs, < 0 on error
int batch_poll(qp_batch* bt)
{
    const hipError_t q = bt->done ? hipEventQuery(bt->done) : hipStreamQuery(bt->stream);
    if (q == hipSuccess) return 1;
    if (q == hipErrorNotReady) return 0;
    return fail(QP_ERR_DEVICE, std::string("batch solve failed: ") + hipGetErrorString(q));
}

void batch_info(const qp_batch* bt, int64_t i, qp_info* info)
{
    const BatchOut& o = bt->out[i];
    std::memset(info, 0, sizeof(*info));
    info->status = o.status;
    info->precision = bt->B.aval32 ? QP_PRECISION_MIXED : QP_PRECISION_FP64;
    info->iterations = o.iterations;
    info->restarts = o.restarts;
    info->inner_iterations = o.inner_iterations;
    info->r_primal = o.r_primal;
    info->r_dual = o.r_dual;
    info->r_gap = o.r_gap;
    info->primal_obj = o.pobj;
    info->dual_obj = o.dobj;
    info->omega = o.omega;
    info->norm_A = bt->norm_A[i];
    info->solve_seconds = bt->solve_seconds;
    info->setup_seconds = bt->setup_seconds;
}

int batch_results_all(qp_batch* bt, std::vector<double>& x, std::vector<double>& y)
{
    if (!bt->solved) return fail(QP_ERR_STATE, "no solve has run on this batch");
    bool pinf = false, dinf = false;
    for (const BatchOut& o : bt->out) {
        pinf |= o.status == QP_PRIMAL_INFEASIBLE;
        dinf |= o.status == QP_DUAL_INFEASIBLE;
    }
    x.resize(bt->n);
    y.resize(bt->m);
    std::vector<double> d, yl;
    HIPCHK(hipMemcpyAsync(x.data(), bt->B.xt, sizeof(double) * bt->n, hipMemcpyDeviceToHost, bt->stream));
    if (bt->m) HIPCHK(hipMemcpyAsync(y.data(), bt->B.yt, sizeof(double) * bt->m, hipMemcpyDeviceToHost, bt->stream));
    if (dinf) {
        d.resize(bt->n);
        HIPCHK(hipMemcpyAsync(d.data(), bt->B.d, sizeof(double) * bt->n, hipMemcpyDeviceToHost, bt->stream));
    }
    if (pinf && bt->m) {
        yl.resize(bt->m);
        HIPCHK(hipMemcpyAsync(yl.data(), bt->B.ytil, sizeof(double) * bt->m, hipMemcpyDeviceToHost, bt->stream));
    }
    HIPCHK(hipStreamSynchronize(bt->stream));
    for (int64_t i = 0; i < bt->count; ++i) {
        const BatchOut& o = bt->out[i];
        if (o.status == QP_DUAL_INFEASIBLE)
            for (int64_t k = bt->voff[i]; k < bt->voff[i + 1]; ++k) x[k] = d[k] / o.d_max;
        if (o.status == QP_PRIMAL_INFEASIBLE)
            for (int64_t k = bt->roff[i]; k < bt->roff[i + 1]; ++k) y[k] = yl[k] / o.ytil_max;
    }
    return 0;
}

// waits for the launched solve and fetches the per-instance outcomes;
// returns the number of OPTIMAL instances
int batch_finish(qp_batch* bt)
{
    HIPCHK(bt->done ? hipEventSynchronize(bt->done) : hipStreamSynchronize(bt->stream));
    bt->solve_seconds = now_s() - bt->t_launch;
    bt->out.resize(bt->count);
    HIPCHK(copy_wait(bt->out.data(), bt->B.out, sizeof(BatchOut) * bt->count, hipMemcpyDeviceToHost, bt->stream));
    bt->solved = 1;
    int opt = 0;
    for (const BatchOut& o : bt->out) opt += o.status == QP_OPTIMAL;
    return opt;
}

}  // namespace pdhcg

extern "C" {

int qp_batch_solve(qp_batch* bt, const qp_params* params)
{
    int rc = batch_launch(bt, params);
    if (rc < 0) return rc;
    rc = batch_finish(bt);
    if (rc >= 0) g_err.clear();
    return rc;
}

int qp_batch_num_shapes(void)
{
    int count = 0;
    pdhcg::batch_shapes(&count);
    return count;
}

int qp_batch_default_shape(int32_t general)
{
    return general ? pdhcg::BATCH_SHAPE_GENERAL_DEFAULT : pdhcg::BATCH_SHAPE_DEFAULT;
}

int qp_batch_shape_info(int32_t shape, int32_t* threads, int32_t* lds_doubles, int32_t* waves_per_simd)
{
    int count = 0;
    const pdhcg::BatchShape* tab = pdhcg::batch_shapes(&count);
    if (shape < 0 || shape >= count) return fail(QP_ERR_INVALID_ARG, "no such batch shape");
    if (threads) *threads = tab[shape].threads;
    if (lds_doubles) *lds_doubles = tab[shape].lds;
    if (waves_per_simd) *waves_per_simd = tab[shape].waves_per_simd;
    return 0;
}

int qp_batch_set_schedule(qp_batch* bt, int32_t shape, int32_t order)
{
    if (!bt) return fail(QP_ERR_INVALID_ARG, "batch is NULL");
    if (shape < -1 || shape >= qp_batch_num_shapes()) return fail(QP_ERR_INVALID_ARG, "no such batch shape");
    if (order < -1 || order > 1) return fail(QP_ERR_INVALID_ARG, "order must be 0, 1 or -1");
    if (shape >= 0) bt->shape = shape;
    if (order >= 0) bt->order = order;
    g_err.clear();
    return 0;
}

int qp_batch_get_schedule(const qp_batch* bt, int32_t* shape, int32_t* order)
{
    if (!bt) return fail(QP_ERR_INVALID_ARG, "batch is NULL");
    if (shape) *shape = bt->shape;
    if (order) *order = bt->order;
    return 0;
}

int qp_batch_tune(qp_batch* bt, const qp_params* params, double* seconds)
{
    if (!bt) return fail(QP_ERR_INVALID_ARG, "batch is NULL");
    const int ns = qp_batch_num_shapes();
    int best = -1;
    double tbest = INFINITY;
    for (int c = 0; c < 2 * ns; ++c) {
        bt->shape = c / 2;
        bt->order = c % 2;
        const int rc = qp_batch_solve(bt, params);
        if (rc < 0) return rc;
        if (seconds) seconds[c] = bt->solve_seconds;
        if (bt->solve_seconds < tbest) { tbest = bt->solve_seconds; best = c; }
    }
    bt->shape = best / 2;
    bt->order = best % 2;
    // leave the batch holding the chosen schedule's results
    const int rc = qp_batch_solve(bt, params);
    if (rc < 0) return rc;
    g_err.clear();
    return best;
}

int qp_batch_result(const qp_batch* bt, int64_t i, double* x, double* y, qp_info* info)
{
    if (!bt || i < 0 || i >= bt->count) return fail(QP_ERR_INVALID_ARG, "bad batch or index");
    if (!bt->solved) return fail(QP_ERR_STATE, "no solve has run on this batch");
    const BatchOut& o = bt->out[i];
    const int64_t v0 = bt->voff[i], n = bt->voff[i + 1] - v0, r0 = bt->roff[i], m = bt->roff[i + 1] - r0;
    if (x) {
        if (o.status == QP_DUAL_INFEASIBLE) {
            HIPCHK(copy_wait(x, bt->B.d + v0, sizeof(double) * n, hipMemcpyDeviceToHost, bt->stream));
            for (int64_t k = 0; k < n; ++k) x[k] /= o.d_max;
        } else {
            HIPCHK(copy_wait(x, bt->B.xt + v0, sizeof(double) * n, hipMemcpyDeviceToHost, bt->stream));
        }
    }
    if (y && m > 0) {
        if (o.status == QP_PRIMAL_INFEASIBLE) {
            HIPCHK(copy_wait(y, bt->B.ytil + r0, sizeof(double) * m, hipMemcpyDeviceToHost, bt->stream));
            for (int64_t k = 0; k < m; ++k) y[k] /= o.ytil_max;
        } else {
            HIPCHK(copy_wait(y, bt->B.yt + r0, sizeof(double) * m, hipMemcpyDeviceToHost, bt->stream));
        }
    }
    if (info) pdhcg::batch_info(bt, i, info);
    return o.status;
}

int qp_batch_statuses(const qp_batch* bt, int32_t* status, double* seconds)
{
    if (!bt) return fail(QP_ERR_INVALID_ARG, "batch is NULL");
    if (!bt->solved) return fail(QP_ERR_STATE, "no solve has run on this batch");
    if (status)
        for (int64_t i = 0; i < bt->count; ++i) status[i] = bt->out[i].status;
    if (seconds) *seconds = bt->solve_seconds;
    return 0;
}

int qp_batch_times(const qp_batch* bt, double* start_s, double* end_s)
{
    if (!bt) return fail(QP_ERR_INVALID_ARG, "batch is NULL");
    if (!bt->solved) return fail(QP_ERR_STATE, "no solve has run on this batch");
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        khz <= 0)
        return fail(QP_ERR_DEVICE, "device wall clock rate unavailable");
    unsigned long long t0 = ~0ull;
    for (const BatchOut& o : bt->out) t0 = std::min(t0, o.t_start);
    const double tick = 1.0 / (1e3 * (double)khz);
    for (int64_t i = 0; i < bt->count; ++i) {
        if (start_s) start_s[i] = (double)(bt->out[i].t_start - t0) * tick;
        if (end_s) end_s[i] = (double)(bt->out[i].t_end - t0) * tick;
    }
    return 0;
}

int64_t qp_spmv_schedule(int64_t rows, const int64_t* rowptr, int32_t* out, int64_t cap)
{
    if (rows < 0 || !rowptr) return fail(QP_ERR_INVALID_ARG, "bad argument");
    std::vector<BlkDesc> blk;
    int nlr = 0, nseg = 0;
    build_plan(rows, rowptr, blk, nlr, nseg);
    if (out)
        for (int64_t i = 0; i < (int64_t)blk.size() && i < cap; ++i) {
            const BlkDesc& b = blk[i];
            const int32_t v[8] = {b.row0, b.nrows, b.k0, b.k1, b.lr, b.seg, b.nseg, b.seg_base};
            std::memcpy(out + 8 * i, v, sizeof(v));
        }
    return (int64_t)blk.size();
}

int qp_norms(const qp_handle* h, double* norm_A, double* norm_Q)
{
    if (!h) return fail(QP_ERR_INVALID_ARG, "handle is NULL");
    if (norm_A) *norm_A = h->norm_A;
    if (norm_Q) *norm_Q = h->norm_Q;
    return 0;
}

}  // extern "C"
