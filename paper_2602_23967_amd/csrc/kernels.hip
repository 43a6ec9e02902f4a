// kernels.hip -- gfx950 kernels of the PDHCG-II hot path.
//
// Every step of the method runs in one of two kernel shapes:
//   k_spmv<E>  row-block CSR SpMV: a block stages up to NNZ_CAP products
//              a_ij * x_j in LDS with coalesced loads of values and column
//              indices, then sums each row with a lane group sized to the
//              block's row count (1..64 lanes, wavefront shuffles), and hands
//              the row sum to the fused epilogue E.  A row longer than NNZ_CAP
//              and at most ROW_PASS_CAP long is one block's strided passes;
//              longer rows are split into segments, each segment block stores
//              its partial sum and a later kernel completes the row in
//              segment order.
//   k_vec<E>   grid-stride elementwise pass with epilogue E.
// A kernel whose epilogue reduces scalars stores one partial per block
// (wavefront xor-shuffle tree, then LDS across the block's 4 waves), and a
// one-block finishing kernel (k_spmv_fin / k_vec_fin) sums the partials in
// block order and runs E::finalize: the scalar control logic of the method
// (step lengths, inner-solver branch, tolerance, restart, PID, status).  The
// kernel boundary is the only grid-wide synchronisation: no device-scope
// fences or atomics (on gfx950 an agent-scope release writes back the XCD's
// L2, which thousands of blocks cannot afford), and no floating-point
// atomics, so every result is reproducible.
#include <math.h>

#include <type_traits>

#include "device_math.h"
#include "pdhcg_internal.h"

namespace pdhcg {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

template <class E, int NT = TPB>
__device__ __forceinline__ void block_reduce(double (&v)[E::NR > 0 ? E::NR : 1], double* lds)
{
    constexpr int NR = E::NR > 0 ? E::NR : 1;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[j] = rcomb(E::kind(j), v[j], __shfl_xor(v[j], off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NR; ++j) lds[wave * NR + j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            double r = lds[j];
            for (int w = 1; w < NT / 64; ++w) r = rcomb(E::kind(j), r, lds[w * NR + j]);
            v[j] = r;
        }
    }
    __syncthreads();
}

struct SumOne {
    static constexpr int NR = 1;
    __device__ static int kind(int) { return R_SUM; }
};

// sum of src[0, n) in exactly the order a FIN_T-thread finishing kernel
// takes (strided per-thread sums, then block_reduce<SumOne, FIN_T>), with
// TPB threads each standing in for FIN_T / TPB of those; the result is
// valid on thread 0.  lds: at least FIN_T / 64 doubles.
__device__ __forceinline__ double sum_in_fin_order(const double* src, int n, double* lds)
{
    constexpr int V = FIN_T / TPB;
    static_assert(FIN_T % TPB == 0, "the finishing block is a multiple of TPB threads");
    double v[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        double a = 0.0;
        for (int i = threadIdx.x + j * TPB; i < n; i += FIN_T) a += src[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        v[j] = a;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < V; ++j) lds[wave + j * (TPB / 64)] = v[j];
    }
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = lds[0];
        for (int w = 1; w < FIN_T / 64; ++w) r += lds[w];
    }
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// the two kernel shapes
// ---------------------------------------------------------------------------

// One row block (or long-row segment) of a product, with products and sums
// in T.  T = float is the mixed-precision form: FP32 values, the operand the
// epilogue hands out in FP32 (for the iteration's products, the difference
// between the operand and the reference point of the last check), FP32 row
// sums widened to FP64, plus the epilogue's FP64 reference product of the
// row.  Partial sums of column parts and of long-row segments are stored
// without the reference; the passes that complete those rows add it.
template <class E, class T>
__device__ __forceinline__ void spmv_block(const CsrDev& M, const E& e, const T* val, T* prod,
                                           const int* srp, double* lds,
                                           double (&acc)[E::NR > 0 ? E::NR : 1])
{
    constexpr bool F32 = std::is_same<T, float>::value;
    const BlkDesc d = M.blk[blockIdx.x];
    const int cnt = d.k1 - d.k0;
    if (cnt > NNZ_CAP || (d.nrows == 1 && M.nparts == 1 && cnt > 256)) {
        // one row of up to ROW_PASS_CAP nonzeros (or a block that holds one
        // long row only): strided passes of the whole block (no staging, all
        // four waves summing), one block sum, the epilogue on thread 0
        e.template prologue<F32>(lds);
        T ts = T(0);
#pragma unroll 4
        for (int q = threadIdx.x; q < cnt; q += TPB) {
            const int j = M.col[d.k0 + q];
            if constexpr (F32) ts += val[d.k0 + q] * e.xval32(j);
            else ts += val[d.k0 + q] * e.xval(j);
        }
        double s[1] = {(double)ts};
        block_reduce<SumOne>(s, lds);
        if (threadIdx.x == 0) {
            if constexpr (F32) e.row(d.row0, s[0] + e.rowref(d.row0), acc);
            else e.row(d.row0, s[0], acc);
        }
        return;
    }
    {
        int cj[NNZ_CAP / TPB];
        T av[NNZ_CAP / TPB];
#pragma unroll
        for (int i = 0; i < NNZ_CAP / TPB; ++i) {
            const int q = threadIdx.x + i * TPB;
            cj[i] = q < cnt ? M.col[d.k0 + q] : -1;
            av[i] = q < cnt ? val[d.k0 + q] : T(0);
        }
        // work an earlier launch left to this block, before its gathers:
        // its loads overlap the block's own column and value loads
        e.template prologue<F32>(lds);
#pragma unroll
        for (int i = 0; i < NNZ_CAP / TPB; ++i) {
            const int q = threadIdx.x + i * TPB;
            if (cj[i] >= 0) {
                if constexpr (F32) prod[q] = av[i] * e.xval32(cj[i]);
                else prod[q] = av[i] * e.xval(cj[i]);
            }
        }
    }
    __syncthreads();

    if (d.nrows > 0) {
        int G = 64;
        while (G > 1 && G * d.nrows > TPB) G >>= 1;
        const int grp = threadIdx.x / G, lane = threadIdx.x - grp * G;
        const bool partial = M.nparts > 1;
        for (int r = grp; r < d.nrows; r += TPB / G) {
            const int row = d.row0 + r;
            const int a = srp[r], b = srp[r + 1];
            T s = T(0);
            for (int i = a + lane; i < b; i += G) s += prod[i];
            for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
            if (lane == 0) {
                if (partial) M.ypart[(size_t)d.lr * M.rows + row] = (double)s;
                else if constexpr (F32) e.row(row, (double)s + e.rowref(row), acc);
                else e.row(row, (double)s, acc);
            }
        }
    } else if (d.nseg > 0) {
        T ts = T(0);
        for (int q = threadIdx.x; q < cnt; q += TPB) ts += prod[q];
        double s[1] = {(double)ts};
        block_reduce<SumOne>(s, lds);
        if (threadIdx.x == 0) M.seg_part[d.seg_base + d.seg] = s[0];
    }
}

// F32: the mixed-precision form for the iteration's own products (E::BULK)
// when the epilogue asks for it (use32(): a mixed solve, and not a product
// that must be exact, such as the gradient after an expansion step)
template <class E, bool F32>
__global__ __launch_bounds__(TPB) void k_spmv(CsrDev M, E epi, double* partials)
{
    constexpr int NR = E::NR > 0 ? E::NR : 1;
    __shared__ double prodbuf[NNZ_CAP];
    __shared__ int srp[PART_ROWS_CAP + 1];   // the block's row pointers, relative to k0
    __shared__ double lds[NR * (TPB / 64)];
    E e = epi;
    if (e.skip()) return;
    e.init();
    const BlkDesc d = M.blk[blockIdx.x];
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = rid(E::kind(j));
    if (d.nrows > 0) {
        const int* rp = M.rowptr + (size_t)d.lr * (M.rows + 1) + d.row0;
        for (int r = threadIdx.x; r <= d.nrows; r += TPB) srp[r] = rp[r] - d.k0;
    }
    bool f32 = false;
    if constexpr (F32) f32 = e.use32();
    if constexpr (F32) {
        if (f32) spmv_block<E, float>(M, e, M.val32, reinterpret_cast<float*>(prodbuf), srp, lds, acc);
    }
    if (!f32) spmv_block<E, double>(M, e, M.val, prodbuf, srp, lds, acc);

    if constexpr (E::NR > 0) {
        if (M.nparts > 1 || !e.reduce) return;   // the row pass reduces, or nothing does
        block_reduce<E>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < NR; ++j) partials[(size_t)blockIdx.x * NR + j] = acc[j];
        }
    }
}

// row pass of a column-partitioned product: y_i = sum over parts (in part
// order) of the partial row sums, handed to the epilogue
template <class E>
__global__ __launch_bounds__(TPB) void k_rows(CsrDev M, E epi, double* partials)
{
    constexpr int NR = E::NR > 0 ? E::NR : 1;
    __shared__ double lds[NR * (TPB / 64)];
    E e = epi;
    if (e.skip()) return;
    e.init();
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = rid(E::kind(j));
    const long long stride = (long long)gridDim.x * TPB;
#pragma unroll 2
    for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < M.rows; i += stride) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < NPARTS; ++p) s += M.ypart[(size_t)p * M.rows + i];
        if (e.use32()) s += e.rowref((int)i);
        e.row((int)i, s, acc);
    }
    if constexpr (E::NR > 0) {
        if (!e.reduce) return;
        block_reduce<E>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < NR; ++j) partials[(size_t)blockIdx.x * NR + j] = acc[j];
        }
    }
}

// The finishing kernels run E::finalize (the method's scalar control logic)
// on a copy of the control block in LDS: the block reads it with one wide
// parallel load while the partials are summed, thread 0 then takes its
// decisions against LDS instead of a chain of dependent global loads, and
// the block writes the copy back.
constexpr int CTRL_WORDS = (int)(sizeof(Ctrl) / 8);
static_assert(sizeof(Ctrl) % 8 == 0, "Ctrl is copied as 64-bit words");

__device__ __forceinline__ void ctrl_to_lds(const Ctrl* g, unsigned long long* s)
{
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(g);
    for (int i = threadIdx.x; i < CTRL_WORDS; i += blockDim.x) s[i] = src[i];
}

// after a barrier that follows ctrl_to_lds: finalize on the copy (thread 0),
// then every thread writes its words back
template <class E>
__device__ __forceinline__ void finalize_in_lds(const E& e, const double* acc, unsigned long long* s)
{
    if (threadIdx.x == 0) {
        E el = e;
        el.ctrl = reinterpret_cast<Ctrl*>(s);
        el.finalize(acc);
    }
    __syncthreads();
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(e.ctrl);
    for (int i = threadIdx.x; i < CTRL_WORDS; i += blockDim.x) dst[i] = s[i];
}


// An earlier epilogue's finishing step carried into this finishing kernel
// (its partials were kept in their own slots): used when no kernel between
// the two launches reads what that finalize writes, saving one launch.
struct NoPre {
    static constexpr int NR = 0;
    Ctrl* ctrl;
    __device__ static int kind(int) { return R_SUM; }
    __device__ void init() {}
    __device__ void finalize(const double*) const {}
};

template <class Pre>
__device__ __forceinline__ void finish_pre(const Pre& pre, int nblk, const double* partials,
                                           unsigned long long* sctrl)
{
    if constexpr (Pre::NR > 0) {
        __shared__ double ldsp[Pre::NR * (FIN_T / 64)];
        double acc[Pre::NR];
#pragma unroll
        for (int j = 0; j < Pre::NR; ++j) acc[j] = rid(Pre::kind(j));
#pragma unroll 4
        for (int b = threadIdx.x; b < nblk; b += FIN_T) {
#pragma unroll
            for (int j = 0; j < Pre::NR; ++j) acc[j] = rcomb(Pre::kind(j), acc[j], partials[(size_t)b * Pre::NR + j]);
        }
        block_reduce<Pre, FIN_T>(acc, ldsp);
        if (threadIdx.x == 0) {
            // init reads the control values the epilogue's own kernel saw
            // (nothing has changed them since)
            Pre el = pre;
            el.ctrl = reinterpret_cast<Ctrl*>(sctrl);
            el.init();
            el.finalize(acc);
        }
        __syncthreads();
    }
}

// one block: runs a carried epilogue's finishing step, completes the long
// rows (their segment partials summed by a fixed tree, or in segment order
// for rows of few segments), sums the per-block partials in block order,
// and runs the epilogue's finalize
template <class E, class Pre = NoPre>
__global__ __launch_bounds__(FIN_T) void k_spmv_fin(CsrDev M, E epi, const double* partials, Pre pre = Pre{},
                                                    int pre_nblk = 0, const double* pre_partials = nullptr)
{
    constexpr int NR = E::NR > 0 ? E::NR : 1;
    __shared__ double lds[NR * (FIN_T / 64)];
    __shared__ unsigned long long sctrl[CTRL_WORDS];
    E e = epi;
    if (e.skip()) return;
    e.init();
    // e.reduce == 0: only the long rows are completed (no reductions, no
    // finishing step, the control block untouched)
    if constexpr (E::NR > 0) {
        if (e.reduce) {
            ctrl_to_lds(e.ctrl, sctrl);
            finish_pre(pre, pre_nblk, pre_partials, sctrl);
        }
    }
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = rid(E::kind(j));
    {
        // long rows with many segments (a budget row, a dense column), or
        // all of them when they are few: the whole block sums each one's
        // segment partials (fixed tree order)
        __shared__ double lds1[FIN_T / 64];
        for (int lr = 0; lr < M.nlr_coop; ++lr) {
            const int row = M.lr_info[3 * lr], base = M.lr_info[3 * lr + 1], nseg = M.lr_info[3 * lr + 2];
            double part[1] = {0.0};
            for (int i = threadIdx.x; i < nseg; i += FIN_T) part[0] += M.seg_part[base + i];
            block_reduce<SumOne, FIN_T>(part, lds1);
            if (threadIdx.x == 0) {
                double total = part[0];
                if (e.use32()) total += e.rowref(row);
                e.row(row, total, acc);
                e.after_long_row(lr, row);
            }
        }
    }
    {
        // the rest: one thread per row (few segments each), in segment order
        for (int lr = M.nlr_coop + threadIdx.x; lr < M.nlr; lr += FIN_T) {
            const int row = M.lr_info[3 * lr], base = M.lr_info[3 * lr + 1], nseg = M.lr_info[3 * lr + 2];
            double total = 0.0;
            for (int i = 0; i < nseg; ++i) total += M.seg_part[base + i];
            if (e.use32()) total += e.rowref(row);
            e.row(row, total, acc);
            e.after_long_row(lr, row);
        }
    }
    if constexpr (E::NR > 0) {
        if (!e.reduce) return;
#pragma unroll 4
        for (int b = threadIdx.x; b < M.nblk; b += FIN_T) {
#pragma unroll
            for (int j = 0; j < NR; ++j) acc[j] = rcomb(E::kind(j), acc[j], partials[(size_t)b * NR + j]);
        }
        block_reduce<E, FIN_T>(acc, lds);
        finalize_in_lds(e, acc, sctrl);
    }
}

template <class E>
__global__ __launch_bounds__(TPB) void k_vec(long long len, E epi, double* partials)
{
    constexpr int NR = E::NR > 0 ? E::NR : 1;
    __shared__ double lds[NR * (TPB / 64)];
    E e = epi;
    if (e.skip()) return;
    e.init();
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = rid(E::kind(j));
    const long long stride = (long long)gridDim.x * TPB;
#pragma unroll 2
    for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < len; i += stride) e.elem(i, acc);
    if constexpr (E::NR > 0) {
        block_reduce<E>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < NR; ++j) partials[(size_t)blockIdx.x * NR + j] = acc[j];
        }
    }
}

template <class E, class Pre = NoPre>
__global__ __launch_bounds__(FIN_T) void k_vec_fin(int nblk, E epi, const double* partials, Pre pre = Pre{},
                                                   int pre_nblk = 0, const double* pre_partials = nullptr)
{
    constexpr int NR = E::NR > 0 ? E::NR : 1;
    __shared__ double lds[NR * (FIN_T / 64)];
    __shared__ unsigned long long sctrl[CTRL_WORDS];
    E e = epi;
    if (e.skip()) return;
    e.init();
    ctrl_to_lds(e.ctrl, sctrl);
    finish_pre(pre, pre_nblk, pre_partials, sctrl);
    double acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = rid(E::kind(j));
#pragma unroll 4
    for (int b = threadIdx.x; b < nblk; b += FIN_T) {
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = rcomb(E::kind(j), acc[j], partials[(size_t)b * NR + j]);
    }
    block_reduce<E, FIN_T>(acc, lds);
    finalize_in_lds(e, acc, sctrl);
}

// ---------------------------------------------------------------------------
// epilogues
// ---------------------------------------------------------------------------

struct EpiBase {
    // true for the products of the iteration proper (not the checks): these
    // run from the FP32 copy of the matrix when the solve is in mixed precision
    static constexpr bool BULK = false;
    Ctrl* ctrl;
    // 0: nothing reads this launch's reductions (an iteration of the
    // closed-form path between the round's first step and the step before a
    // check), so its kernels leave no partials and no finishing step runs
    int reduce = 1;
    __device__ bool skip() const { return false; }
    __device__ void init() {}
    // mixed precision (BULK epilogues): whether this launch takes the FP32
    // form, the operand it then gathers, and the FP64 reference product of a row
    __device__ bool use32() const { return false; }
    __device__ float xval32(int) const { return 0.0f; }
    __device__ double rowref(int) const { return 0.0; }
    __device__ static int kind(int) { return R_SUM; }
    __device__ void finalize(const double*) const {}
    // work an earlier launch left to every block of this product, run before
    // the block gathers its operand (all threads of the block call it);
    // F32: the block gathers the FP32 operand
    template <bool F32>
    __device__ void prologue(double*) const {}
    // after a finishing kernel completed long row lr (row i)
    __device__ void after_long_row(int, int) const {}
};

template <int N>
using Acc = double (&)[N > 0 ? N : 1];

// decision shared by every point where the inner solver has fresh split
// statistics: stop test (Section 3.3 tolerance), proportioning test, and the
// kind of the next direction
__device__ void inner_decide(Ctrl* c, double gp2, double b2, double ptp, long long seq,
                             unsigned long long* dstat)
{
    c->gp2 = gp2; c->b2 = b2; c->ptp = ptp;
    c->res = sqrt(gp2);
    const double eps = c->eps_fixed > 0.0 ? c->eps_fixed : c->eps;
    c->done = (c->res <= eps || c->inner_it >= c->max_inner) ? 1 : 0;
    const int prop = b2 <= c->mprgp_gamma * c->mprgp_gamma * ptp;
    c->proportional = prop;
    c->dir_mode = !prop ? DIR_BETA : (c->last_step == STEP_CG ? DIR_CONJ : DIR_PHI);
    post_status(dstat, seq, c->done);
}

// dual step (eq. dual_update) on the extrapolated point x_bar = 2 x_T - x
// (eq. extrapolation), then the reflected Halpern average of y (Section 3.1)
struct EpiDual : EpiBase {
    static constexpr bool BULK = true;
    static constexpr int NR = 4;
    const double *xbar, *ya, *lc, *uc;
    double *y, *yt, *ytil;
    int store;
    // mixed precision: A x_bar = A x_ref + A(x_bar - x_ref) (dxb32, axref), and
    // y - y_ref is written for the next primal step's product
    const float* dxb32 = nullptr;
    const double *axref = nullptr, *yref = nullptr;
    float* dy32 = nullptr;
    __device__ bool use32() const { return dxb32 != nullptr; }
    __device__ float xval32(int j) const { return dxb32[j]; }
    __device__ double rowref(int i) const { return axref[i]; }
    double sigma, w, wa, th;
    int halpern;
    // >= 0: the iteration count k and the round's step count t, given by the
    // host (the closed-form path), else read from ctrl
    long long tk = -1, kk = -1;
    // closed-form path, A with long rows: y of the long rows after this
    // step, in the slot of this iteration's parity (a step that leaves its
    // long rows to the next primal kernel reads the other slot there)
    double* ylr_out = nullptr;
    __device__ static int kind(int j) { return j == 1 ? R_MAX : R_SUM; }
    __device__ void init()
    {
        sigma = ctrl->sigma;
        const double t = (double)(tk >= 0 ? tk : ctrl->t);
        w = (t + 1.0) / (t + 2.0);
        wa = 1.0 / (t + 2.0);
        th = ctrl->theta;
        halpern = ctrl->use_halpern;
    }
    __device__ double xval(int j) const { return xbar[j]; }
    // the dual step of a row from its product s, the previous y_i, the
    // row's bounds and anchor: returns the new y_i (Halpern average) and y_T,i
    // in yti
    __device__ double step_v(double s, double yi, double l, double u, double yai, double& yti) const
    {
        const double v = yi / sigma + s;
        yti = sigma * (v - clampd(v, l, u));
        return halpern ? w * ((1.0 + th) * yti - th * yi) + wa * yai : yti;
    }
    __device__ double step(int i, double s, double yi, double& yti) const
    {
        return step_v(s, yi, lc[i], uc[i], ya[i], yti);
    }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double yi = y[i];
        double yti;
        const double yn = step(i, s, yi, yti);
        const double dy = yti - yi;
        a[0] += dy * dy;
        yt[i] = yti;
        y[i] = yn;
        if (dy32) dy32[i] = (float)(yn - yref[i]);
        if (store) {
            const double yy = projY(dy, lc[i], uc[i]);
            ytil[i] = yy;
            a[1] = rcomb(R_MAX, a[1], fabs(yy));
            a[2] += supp(yy, lc[i], uc[i]);
            a[3] += supp_abs(yy, lc[i], uc[i]);
        }
    }
    __device__ void after_long_row(int lr, int i) const
    {
        if (ylr_out) ylr_out[lr] = y[i];
    }
    // long row lr (row i) of a step that left its long rows to the next
    // primal kernel, completed there by every block: the previous y_i comes
    // from the copy kept by the previous completion (y itself may already
    // hold this step's value, stored by another block); every block stores
    // y_i and its FP32 difference (the same values) before it gathers them,
    // block 0 also y_T,i and the copy for the next completion.  No
    // reductions: nothing reads them for such a step.
    __device__ void long_row_late(int lr, int i, double s, const double* ylr_in, bool first) const
    {
        double yti;
        const double yn = step(i, s, ylr_in[lr], yti);
        store_late(lr, i, yn, yti, dy32 ? yref[i] : 0.0, first);
    }
    __device__ void store_late(int lr, int i, double yn, double yti, double yrefi, bool first) const
    {
        y[i] = yn;
        if (dy32) dy32[i] = (float)(yn - yrefi);
        if (first) {
            yt[i] = yti;
            ylr_out[lr] = yn;
        }
    }
    // the last kernel of an iteration: the counters advance here, and the
    // residual of the round's first step is kept for the restart test
    __device__ void finalize(const double* t) const
    {
        Ctrl* C = ctrl;
        C->ndy2 = t[0];
        if (store) {
            C->ytil_max = t[1];
            C->ptil_sum = t[2];
            C->ptil_abs = t[3];
        }
        if (tk >= 0) {
            C->k = kk + 1;
            C->t = tk + 1;
        } else {
            C->k += 1;
            C->t += 1;
        }
        if (C->t == 1) C->R_start = sqrt(C->omega * C->ndx2 + C->ndy2 / C->omega);
    }
};


// Reflected Halpern average of x (Section 3.1) for one row, fused into the
// kernel that produces x_T: x <- w((1+theta) x_T - theta x) + wa x_anchor,
// the movement ||x_T - x||^2 and, when a check follows, the pieces of the
// unboundedness certificate d = proj_Recc(X)(x_T - x) (Section 5).
struct HalpernX {
    const double *xa, *c;
    BoundVec lv, uv;
    double *x, *d;
    int store;
    double w, wa, th;
    int halpern, unb;
    long long tk = -1;   // >= 0: the round's step count t, given by the host (else ctrl->t)
    __device__ void init(const Ctrl* ctrl)
    {
        const double t = (double)(tk >= 0 ? tk : ctrl->t);
        w = (t + 1.0) / (t + 2.0);
        wa = 1.0 / (t + 2.0);
        th = ctrl->theta;
        halpern = ctrl->use_halpern;
        unb = ctrl->has_unbounded_x;
    }
    __device__ void row(long long i, double xti, double xi, double (&a)[3]) const
    {
        const double dxi = xti - xi;
        a[0] += dxi * dxi;
        x[i] = halpern ? w * ((1.0 + th) * xti - th * xi) + wa * xa[i] : xti;
        if (store && unb) {
            const double di = projRec(dxi, lv[i], uv[i]);
            d[i] = di;
            a[1] = rcomb(R_MAX, a[1], fabs(di));
            a[2] += c[i] * di;
        }
    }
    // movement, certificate pieces and the inner-tolerance update (Section
    // 3.3); the iteration counters advance after the dual step
    __device__ void finalize(Ctrl* C, const double* t) const
    {
        C->ndx2 = t[0];
        if (store) {
            C->d_max = unb ? t[1] : 0.0;
            C->cd = unb ? t[2] : 0.0;
        }
        if (C->eps_fixed <= 0.0)
            C->eps = fmin(C->eps, fmax(C->gamma_inner * C->omega * sqrt(t[0]) / C->tau, C->eps_min));
    }
};

// primal step, diagonal Q (Section 2.2 closed form), fused into A'y:
//   x_T = clip((x/tau - c - A'y) / (q + 1/tau), l_v, u_v)
struct EpiProx : EpiBase {
    static constexpr bool BULK = true;
    static constexpr int NR = 3;
    const double *y, *c, *qd;
    BoundVec lv, uv;
    double *x, *xt, *xbar;
    HalpernX hx;
    // mixed precision: A' y = A' y_ref + A'(y - y_ref) (dy32, aty_ref), and
    // x_bar - x_ref is written for the dual step's product
    const float* dy32 = nullptr;
    const double *atyref = nullptr, *xref = nullptr;
    float* dxb32 = nullptr;
    double it;
    // lr_n > 0: the previous dual step (lrd) left its long rows to this
    // kernel (an iteration whose reductions nothing reads: its one-block
    // finishing kernel, which would only have completed them, did not run).
    // Every block completes them from their segment partials, summed in the
    // finishing kernel's order, before it gathers y.
    EpiDual lrd;
    const int* lr_info = nullptr;      // A's long rows: {row, first segment slot, segment count}
    const double* lr_seg = nullptr;    // A's segment partials
    const double* ylr_in = nullptr;    // y of the long rows before that step
    int lr_n = 0, lr_coop = 0;
    int lr0[3] = {-1, 0, 0};           // lr_info of long row 0 (one of the block-summed rows)
    // mixed precision: long row 0's FP32 difference y - y_ref, held by every
    // thread of the block, which gathers it from here (the FP32 product
    // gathers nothing else of y), so only block 0 stores that row's values;
    // a store from every block into the line the others gather from cost
    // the mixed kernel 1.6 % of a solve.  FP64 gathers y itself: there every
    // block stores the row's new y (a select per gather measured slower).
    int lr0_live = -1;
    mutable float lr0_d32 = 0.0f;
    __device__ static int kind(int j) { return j == 1 ? R_MAX : R_SUM; }
    __device__ void init()
    {
        it = ctrl->inv_tau;
        hx.init(ctrl);
        if (lr_n > 0) lrd.init();
        lr0_live = (lr_n > 0 && lr_coop > 0 && lrd.dy32 != nullptr) ? lr0[0] : -1;
    }
    template <bool F32>
    __device__ void prologue(double* lds) const
    {
        static_assert(NR * (TPB / 64) >= FIN_T / 64 + 1,
                      "k_spmv's reduction buffer holds the ordered sum and long row 0's value");
        if (lr_n == 0) return;
        const bool keep0 = F32 && lr0_live >= 0;   // long row 0's FP32 value kept in registers
        const bool first = blockIdx.x == 0;
        if (lr_coop > 0) {
            // long row 0 (a budget row, a dense row): its own values are
            // loaded while its segment partials are summed
            const int row = lr0[0];
            double l = 0.0, u = 0.0, yai = 0.0, yi = 0.0, ref = 0.0, yrefi = 0.0;
            if (threadIdx.x == 0) {
                l = lrd.lc[row];
                u = lrd.uc[row];
                yai = lrd.ya[row];
                yi = ylr_in[0];
                if (lrd.use32()) {
                    ref = lrd.rowref(row);
                    yrefi = lrd.yref[row];
                }
            }
            const double part = sum_in_fin_order(lr_seg + lr0[1], lr0[2], lds);
            if (threadIdx.x == 0) {
                double total = part;
                if (lrd.use32()) total += ref;
                double yti;
                const double yn = lrd.step_v(total, yi, l, u, yai, yti);
                if (first || !keep0) lrd.store_late(0, row, yn, yti, yrefi, first);
                if (keep0) lds[FIN_T / 64] = (double)(float)(yn - yrefi);
            }
        }
        for (int lr = 1; lr < lr_coop; ++lr) {
            const int row = lr_info[3 * lr], base = lr_info[3 * lr + 1], nseg = lr_info[3 * lr + 2];
            const double part = sum_in_fin_order(lr_seg + base, nseg, lds);
            if (threadIdx.x == 0) {
                double total = part;
                if (lrd.use32()) total += lrd.rowref(row);
                lrd.long_row_late(lr, row, total, ylr_in, first);
            }
        }
        for (int lr = lr_coop + threadIdx.x; lr < lr_n; lr += TPB) {
            const int row = lr_info[3 * lr], base = lr_info[3 * lr + 1], nseg = lr_info[3 * lr + 2];
            double total = 0.0;
            for (int i = 0; i < nseg; ++i) total += lr_seg[base + i];
            if (lrd.use32()) total += lrd.rowref(row);
            lrd.long_row_late(lr, row, total, ylr_in, first);
        }
        __syncthreads();
        if (keep0) lr0_d32 = (float)lds[FIN_T / 64];
    }
    __device__ double xval(int j) const { return y[j]; }
    __device__ bool use32() const { return dy32 != nullptr; }
    __device__ float xval32(int j) const { return j == lr0_live ? lr0_d32 : dy32[j]; }
    __device__ double rowref(int i) const { return atyref[i]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double xi = x[i];
        const double v = clampd((xi * it - c[i] - s) / (qd[i] + it), lv[i], uv[i]);
        xt[i] = v;
        const double xb = 2.0 * v - xi;
        xbar[i] = xb;
        if (dxb32) dxb32[i] = (float)(xb - xref[i]);
        hx.row(i, v, xi, a);
    }
    __device__ void finalize(const double* t) const { hx.finalize(ctrl, t); }
};

// extrapolated point x_bar = 2 x_T - x (eq. extrapolation) and the Halpern
// average of x
struct EpiXbar : EpiBase {
    static constexpr int NR = 3;
    const double* xt;
    double* xbar;
    HalpernX hx;
    const double* xref = nullptr;   // mixed precision: also x_bar - x_ref in FP32
    float* dxb32 = nullptr;
    __device__ static int kind(int j) { return j == 1 ? R_MAX : R_SUM; }
    __device__ void init() { hx.init(ctrl); }
    __device__ void elem(long long i, Acc<NR> a) const
    {
        const double xti = xt[i], xi = hx.x[i];
        const double xb = 2.0 * xti - xi;
        xbar[i] = xb;
        if (dxb32) dxb32[i] = (float)(xb - xref[i]);
        hx.row(i, xti, xi, a);
    }
    __device__ void finalize(const double* t) const { hx.finalize(ctrl, t); }
};

// x <- clip(x, l_v, u_v)
struct EpiClip : EpiBase {
    static constexpr int NR = 0;
    BoundVec lv, uv;
    double* x;
    __device__ void elem(long long i, Acc<NR>) const { x[i] = clampd(x[i], lv[i], uv[i]); }
};

// rhs of the primal subproblem (eq. primal_update): rhs = x/tau - c - A'y
struct EpiRhs : EpiBase {
    static constexpr bool BULK = true;
    static constexpr int NR = 0;
    const double *y, *x, *c;
    double* rhs;
    const float* dy32 = nullptr;
    const double* atyref = nullptr;
    double it;
    __device__ void init() { it = ctrl->inv_tau; }
    __device__ double xval(int j) const { return y[j]; }
    __device__ bool use32() const { return dy32 != nullptr; }
    __device__ float xval32(int j) const { return dy32[j]; }
    __device__ double rowref(int i) const { return atyref[i]; }
    __device__ void row(int i, double s, Acc<NR>) const { rhs[i] = x[i] * it - c[i] - s; }
};

// rhs of the new subproblem and its gradient at the warm start x_T without a
// product with Q: the previous subproblem ended with g = Q x_T + x_T/tau' - rhs'
// (tau', rhs' its step and right-hand side), so the new gradient is
// g + (rhs' - rhs) + x_T (1/tau - 1/tau'); split statistics as in EpiGinit
struct EpiRhsGrad : EpiBase {
    static constexpr bool BULK = true;
    static constexpr int NR = 3;
    const double *y, *x, *c, *xt;
    BoundVec lv, uv;
    double *rhs, *g;
    unsigned long long* dstat;
    long long seq;
    const float* dy32 = nullptr;
    const double* atyref = nullptr;
    __device__ bool use32() const { return dy32 != nullptr; }
    __device__ float xval32(int j) const { return dy32[j]; }
    __device__ double rowref(int i) const { return atyref[i]; }
    double it, dit, abar;
    __device__ void init()
    {
        it = ctrl->inv_tau;
        dit = ctrl->inv_tau - ctrl->g_inv_tau;
        abar = ctrl->abar;
    }
    __device__ double xval(int j) const { return y[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double r = x[i] * it - c[i] - s;
        const double xi = xt[i];
        const double gi = g[i] + (rhs[i] - r) + xi * dit;
        rhs[i] = r;
        g[i] = gi;
        const Split sp = split(xi, gi, lv[i], uv[i], abar);
        a[0] += sp.phi * sp.phi + sp.beta * sp.beta;
        a[1] += sp.beta * sp.beta;
        a[2] += sp.phit * sp.phi;
    }
    __device__ void finalize(const double* t) const
    {
        Ctrl* c = ctrl;
        c->inner_it = 0;
        c->last_step = STEP_NONE;
        c->need_g = 0;
        c->skip_update = 0;
        c->g_inv_tau = c->inv_tau;
        c->seq_base = seq;
        c->step = 0;
        inner_decide(c, t[0], t[1], t[2], seq, dstat);
    }
};

// gradient of the subproblem at the warm start (feasible): g = Q x + x/tau - rhs,
// with split statistics; finalize starts the inner solve
struct EpiGinit : EpiBase {
    static constexpr int NR = 3;   // the exact gradient: FP64 in every precision
    const double* xt;
    const double* rhs;
    BoundVec lv, uv;
    double* g;
    unsigned long long* dstat;
    long long seq;
    double it, abar;
    __device__ void init() { it = ctrl->inv_tau; abar = ctrl->abar; }
    __device__ double xval(int j) const { return xt[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double xi = xt[i];
        const double gi = s + it * xi - rhs[i];
        g[i] = gi;
        const Split sp = split(xi, gi, lv[i], uv[i], abar);
        a[0] += sp.phi * sp.phi + sp.beta * sp.beta;
        a[1] += sp.beta * sp.beta;
        a[2] += sp.phit * sp.phi;
    }
    __device__ void finalize(const double* t) const
    {
        Ctrl* c = ctrl;
        c->inner_it = 0;
        c->last_step = STEP_NONE;
        c->need_g = 0;
        c->skip_update = 0;
        c->g_inv_tau = c->inv_tau;
        if (isinf(c->eps) && c->eps_fixed <= 0.0) c->eps = fmax(c->gamma_inner * sqrt(t[0]), c->eps_min);
        c->seq_base = seq;
        c->step = 0;
        inner_decide(c, t[0], t[1], t[2], seq, dstat);
    }
};

// inner step, part A: H p = Q p + p/tau with p'Hp, g'p and the feasible
// step; or, right after an expansion step, the fresh gradient g = H x - rhs
template <int BM>   // BoundVec storage mode of the box
struct EpiStepA : EpiBase {
    static constexpr bool BULK = true;
    static constexpr int NR = 4;
    const double* __restrict__ p;
    const double* __restrict__ rhs;
    BoundVec lv, uv;
    double* __restrict__ xt;
    double* __restrict__ g;
    double* __restrict__ hp;
    unsigned long long* dstat;
    double it, abar;
    int ng;
    int mixed = 0;   // mixed precision: H p in FP32; the gradient after an expansion stays FP64
    __device__ bool use32() const { return mixed && !ng; }
    __device__ float xval32(int j) const { return (float)p[j]; }
    __device__ static int kind(int j) { return j == 3 ? R_MIN : R_SUM; }
    __device__ bool skip() const { return ctrl->done != 0; }
    __device__ void init() { it = ctrl->inv_tau; abar = ctrl->abar; ng = ctrl->need_g; }
    __device__ double xval(int j) const { return ng ? xt[j] : p[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double l = lv.template at<BM>(i), u = uv.template at<BM>(i);
        if (ng) {
            const double xi = xt[i], ri = rhs[i];
            const double gi = s + it * xi - ri;
            g[i] = gi;
            const Split sp = split(xi, gi, l, u, abar);
            a[0] += sp.phi * sp.phi + sp.beta * sp.beta;
            a[1] += sp.beta * sp.beta;
            a[2] += sp.phit * sp.phi;
        } else {
            // every load first, then the arithmetic and the store
            const double pi = p[i], xi = xt[i], gi = g[i];
            const double h = s + it * pi;
            hp[i] = h;
            a[0] += pi * h;
            a[1] += gi * pi;
            double st = INFINITY;
            if (pi > 0.0 && isfinite(l)) st = (xi - l) / pi;
            else if (pi < 0.0 && isfinite(u)) st = (xi - u) / pi;
            a[3] = fmin(a[3], st);
        }
    }
    __device__ void finalize(const double* t) const
    {
        Ctrl* c = ctrl;
        c->hp_active += 1;
        c->step += 1;   // every inner step that is not past the stop runs this
        const long long seq = c->seq_base + c->step;
        if (ng) {
            c->need_g = 0;
            c->skip_update = 1;
            inner_decide(c, t[0], t[1], t[2], seq, dstat);
            return;
        }
        c->skip_update = 0;
        const double pHp = t[0], gp = t[1];
        double af = t[3] < 0.0 ? 0.0 : t[3];
        if (!(pHp > 0.0)) {   // no descent direction left: stop
            c->done = 1;
            c->skip_update = 1;
            post_status(dstat, seq, 1);
            return;
        }
        c->pHp = pHp;
        const double acg = gp / pHp;
        if (c->dir_mode == DIR_BETA) {
            c->step_kind = STEP_PROP;
            c->alpha = acg < af ? acg : af;
        } else if (acg <= af) {
            c->step_kind = STEP_CG;
            c->alpha = acg;
        } else {
            c->step_kind = STEP_EXPAND;
            c->alpha = af;
        }
    }
};

// inner step, part B: x <- clip(x - alpha p), g <- g - alpha Hp; expansion
// adds the projected step x <- clip(x - abar phi(x)) and asks for a fresh g
template <int BM>
struct EpiStepB : EpiBase {
    static constexpr int NR = 4;
    const double* __restrict__ p;
    const double* __restrict__ hp;
    BoundVec lv, uv;
    double* __restrict__ xt;
    double* __restrict__ g;
    unsigned long long* dstat;
    double alpha, abar;
    int kindstep;
    __device__ bool skip() const { return ctrl->done != 0 || ctrl->skip_update != 0; }
    __device__ void init() { alpha = ctrl->alpha; abar = ctrl->abar; kindstep = ctrl->step_kind; }
    __device__ void elem(long long i, Acc<NR> a) const
    {
        const double l = lv.template at<BM>(i), u = uv.template at<BM>(i);
        const double x0 = xt[i], pi = p[i], g0 = g[i], hi = hp[i];
        double xi = clampd(x0 - alpha * pi, l, u);
        const double gi = g0 - alpha * hi;
        g[i] = gi;
        const Split sp = split(xi, gi, l, u, abar);
        if (kindstep == STEP_EXPAND) {
            xi = clampd(xi - abar * sp.phi, l, u);
        } else {
            a[0] += sp.phi * sp.phi + sp.beta * sp.beta;
            a[1] += sp.beta * sp.beta;
            a[2] += sp.phit * sp.phi;
            a[3] += sp.phi * hi;
        }
        xt[i] = xi;
    }
    __device__ void finalize(const double* t) const
    {
        Ctrl* c = ctrl;
        c->inner_it += 1;
        c->inner_total += 1;
        const long long seq = c->seq_base + c->step;
        if (kindstep == STEP_EXPAND) {
            c->last_step = STEP_EXPAND;
            c->need_g = 1;
            post_status(dstat, seq, 0);
            return;
        }
        if (kindstep == STEP_CG) c->gam = t[3] / c->pHp;
        c->last_step = kindstep;
        inner_decide(c, t[0], t[1], t[2], seq, dstat);
    }
};

// next direction: beta (proportioning), phi, or phi - gam p (conjugate)
template <int BM>
struct EpiDir : EpiBase {
    static constexpr int NR = 0;
    const double* __restrict__ xt;
    const double* __restrict__ g;
    BoundVec lv, uv;
    double* __restrict__ p;
    double gam, abar;
    int mode;
    __device__ bool skip() const { return ctrl->done != 0 || ctrl->need_g != 0; }
    __device__ void init() { gam = ctrl->gam; abar = ctrl->abar; mode = ctrl->dir_mode; }
    __device__ void elem(long long i, Acc<NR>) const
    {
        const double pi = p[i];
        const Split sp = split(xt[i], g[i], lv.template at<BM>(i), uv.template at<BM>(i), abar);
        p[i] = mode == DIR_BETA ? sp.beta : (mode == DIR_PHI ? sp.phi : sp.phi - gam * pi);
    }
};

// ---- Q = P + R'R given by its factors (Section 2.2) -------------------------
// A product with Q is a product with the n x (n + k) matrix [P | R'] on the
// operand [v; R v]: the k entries R v live right after the operand's n
// entries.  These epilogues compute that tail.

// tail = R v (Bulk: part of the iteration, FP32 in mixed precision)
template <bool Bulk>
struct EpiTail : EpiBase {
    static constexpr bool BULK = Bulk;
    static constexpr int NR = 0;
    const double* v;
    double* tail;
    __device__ double xval(int j) const { return v[j]; }
    __device__ void row(int r, double s, Acc<NR>) const { tail[r] = s; }
};

// the tail of the inner step's operand: R p, or R x right after an expansion
struct EpiTailHp : EpiBase {
    static constexpr bool BULK = true;
    static constexpr int NR = 0;
    const double *p, *xt;
    double *ptail, *xtail;
    int ng;
    int mixed = 0;
    __device__ bool use32() const { return mixed && !ng; }
    __device__ float xval32(int j) const { return (float)p[j]; }
    __device__ bool skip() const { return ctrl->done != 0; }
    __device__ void init() { ng = ctrl->need_g; }
    __device__ double xval(int j) const { return ng ? xt[j] : p[j]; }
    __device__ void row(int r, double s, Acc<NR>) const { (ng ? xtail : ptail)[r] = s; }
};

// ---- check kernels (Sections 4 and 5) -------------------------------------

// w = A' ytil: violation of A'ytil in R and p(-proj_R(A'ytil); l_v, u_v)
struct EpiPinf : EpiBase {
    static constexpr int NR = 3;
    const double* ytil;
    BoundVec lv, uv;
    __device__ static int kind(int j) { return j == 0 ? R_MAX : R_SUM; }
    __device__ double xval(int j) const { return ytil[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double wh = projR(s, lv[i], uv[i]);
        a[0] = rcomb(R_MAX, a[0], fabs(s - wh));
        a[1] += supp(-wh, lv[i], uv[i]);
        a[2] += supp_abs(-wh, lv[i], uv[i]);
    }
    __device__ void finalize(const double* t) const
    {
        ctrl->w_viol = t[0];
        ctrl->pw_sum = t[1];
        ctrl->pw_abs = t[2];
    }
};

// A d: violation of A d in Recc(S)
struct EpiAd : EpiBase {
    static constexpr int NR = 1;
    const double *d, *lc, *uc;
    __device__ static int kind(int) { return R_MAX; }
    __device__ double xval(int j) const { return d[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        a[0] = rcomb(R_MAX, a[0], fabs(s - projRec(s, lc[i], uc[i])));
    }
    __device__ void finalize(const double* t) const { ctrl->ad_viol = t[0]; }
};

// Q d: its largest magnitude
struct EpiQd : EpiBase {
    static constexpr int NR = 1;
    const double* d;
    __device__ static int kind(int) { return R_MAX; }
    __device__ double xval(int j) const { return d[j]; }
    __device__ void row(int, double s, Acc<NR> a) const { a[0] = rcomb(R_MAX, a[0], fabs(s)); }
    __device__ void finalize(const double* t) const { ctrl->qd_max = t[0]; }
};

// A' y written out, with ||A'y||_inf
struct EpiAty : EpiBase {
    static constexpr int NR = 1;
    const double* y;
    double* aty;
    double* atyref = nullptr;   // mixed precision: the reference product A' y_T
    __device__ static int kind(int) { return R_MAX; }
    __device__ double xval(int j) const { return y[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        aty[i] = s;
        if (atyref) atyref[i] = s;
        a[0] = rcomb(R_MAX, a[0], fabs(s));
    }
    __device__ void finalize(const double* t) const { ctrl->aty_max = t[0]; }
};

// A x: primal violation, p(y; l_c, u_c), and the dual movement of the round
struct EpiAx : EpiBase {
    static constexpr int NR = 3;
    const double *x, *y, *ya, *lc, *uc;
    double* axref = nullptr;   // mixed precision: the reference product A x_T
    __device__ static int kind(int j) { return j == 0 ? R_MAX : R_SUM; }
    __device__ double xval(int j) const { return x[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        if (axref) axref[i] = s;
        const double l = lc[i], u = uc[i], yi = y[i];
        a[0] = rcomb(R_MAX, a[0], fabs(s - clampd(s, l, u)));
        a[1] += supp(yi, l, u);
        if (ya) {
            const double dv = yi - ya[i];
            a[2] += dv * dv;
        }
    }
    __device__ void finalize(const double* t) const
    {
        ctrl->pviol = t[0];
        ctrl->py_sum = t[1];
        ctrl->mvy2 = t[2];
    }
};

__device__ bool primal_infeasible(const Ctrl* c)
{
    if (!(c->ytil_max > 0.0) || !isfinite(c->ytil_max)) return false;
    const double val = c->pw_sum + c->ptil_sum;
    const double imp = val < 0.0 ? -val : 0.0;
    const double mag = c->pw_abs + c->ptil_abs;
    return imp > 1e-9 * mag && c->w_viol <= c->eps_inf * imp;
}

__device__ bool dual_infeasible(const Ctrl* c)
{
    if (!c->has_unbounded_x || !(c->d_max > 0.0) || !isfinite(c->d_max)) return false;
    if (!(c->cd / c->d_max < -c->tol)) return false;
    const double v1 = c->ad_viol / c->d_max;
    const double v2 = c->qd_max / c->d_max / c->gamma_q;
    return (v1 > v2 ? v1 : v2) <= c->eps_inf;
}

// Q x with r = Qx + c + A'y: dual violation, norms, objective pieces, gap
// terms, natural residual and the primal movement of the round; when `full`,
// finalize makes the termination / infeasibility / restart decision
struct EpiQx : EpiBase {
    static constexpr int NR = 7;
    const double *x, *xa, *c, *aty;
    BoundVec lv, uv;
    unsigned long long* dcheck;
    int full;
    __device__ static int kind(int j) { return (j == 0 || j == 1 || j == 5) ? R_MAX : R_SUM; }
    __device__ double xval(int j) const { return x[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        const double xi = x[i], l = lv[i], u = uv[i];
        const double r = s + c[i] + aty[i];
        const double rh = projR(r, l, u);
        a[0] = rcomb(R_MAX, a[0], fabs(r - rh));
        a[1] = rcomb(R_MAX, a[1], fabs(s));
        a[2] += xi * s;
        a[3] += c[i] * xi;
        a[4] += supp(-rh, l, u);
        a[5] = rcomb(R_MAX, a[5], fabs(xi - clampd(xi - r, l, u)));
        if (xa) {
            const double dv = xi - xa[i];
            a[6] += dv * dv;
        }
    }
    __device__ void finalize(const double* t) const
    {
        Ctrl* C = ctrl;
        C->dviol = t[0]; C->qx_max = t[1]; C->xqx = t[2]; C->cx = t[3];
        C->pr_sum = t[4]; C->natural = t[5]; C->mvx2 = t[6];
        C->r_primal = C->pviol / C->bscale_p;
        double sd = C->qx_max > C->aty_max ? C->qx_max : C->aty_max;
        sd = sd > C->c_max ? sd : C->c_max;
        C->r_dual = C->dviol / (1.0 + sd);
        C->pobj = 0.5 * C->xqx + C->cx;
        const double dneg = 0.5 * C->xqx + C->pr_sum + C->py_sum;
        C->dobj = -dneg;
        const double gap = fabs(C->xqx + C->cx + C->pr_sum + C->py_sum);
        const double den = fabs(C->pobj) > fabs(dneg) ? fabs(C->pobj) : fabs(dneg);
        C->r_gap = gap / (1.0 + den);
        if (!full) return;

        C->checks += 1;
        double worst = C->r_primal > C->r_dual ? C->r_primal : C->r_dual;
        worst = worst > C->r_gap ? worst : C->r_gap;
        int st = 0, restart = 0;
        if (!isfinite(worst) || worst != worst) st = 5;
        else if (worst <= C->tol) st = 1;
        else if (C->k > 0 && primal_infeasible(C)) st = 2;
        else if (C->k > 0 && dual_infeasible(C)) st = 3;
        else if (C->k >= C->max_iter) st = 4;
        else {
            // restart rule on the weighted fixed-point residual of the last step
            const double R = sqrt(C->omega * C->ndx2 + C->ndy2 / C->omega);
            restart = R <= C->rs_suff * C->R_start ||
                      (C->R_prev_valid && R <= C->rs_nec * C->R_start && R > C->R_prev) ||
                      (double)C->t >= C->rs_art * (double)C->k;
            C->R_prev = R;
            C->R_prev_valid = 1;
            if (restart) {
                // PID on log(omega) over the round (Section 3.2, eq. pid)
                const double mx = sqrt(C->mvx2), my = sqrt(C->mvy2);
                if (mx > 1e-10 && my > 1e-10 && isfinite(mx) && isfinite(my)) {
                    const double so = sqrt(C->omega);
                    const double e = log(so * mx / (my / so));
                    C->pid_int += e;
                    double lw = log(C->omega) - (C->kp * e + C->ki * C->pid_int + C->kd * (e - C->pid_prev));
                    const double lo = log(C->omega0) - 10.0, hi = log(C->omega0) + 10.0;
                    lw = lw < lo ? lo : (lw > hi ? hi : lw);
                    C->omega = exp(lw);
                    C->pid_prev = e;
                }
                C->tau = C->eta / C->omega;
                C->sigma = C->eta * C->omega;
                C->inv_tau = 1.0 / C->tau;
                C->abar = C->abar_scale / (C->norm_Q + C->inv_tau);
                C->t = 0;
                C->R_prev_valid = 0;
                C->restarts += 1;
            }
        }
        C->status = st;
        C->restart_pending = restart;
        C->pinf = st == 2;
        C->dinf = st == 3;
        // the host's view of the decision: check count, restart, stop
        __hip_atomic_store(dcheck,
                           (static_cast<unsigned long long>(C->checks) << 2) | (restart ? 2ull : 0ull) |
                               (st != 0 ? 1ull : 0ull),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
};

// restart: x, anchor <- x_T; y, anchor <- y_T
struct EpiRestart : EpiBase {
    static constexpr int NR = 0;
    const double *xt, *yt;
    double *x, *xa, *y, *ya;
    int n;
    __device__ bool skip() const { return ctrl->restart_pending == 0; }
    __device__ void elem(long long i, Acc<NR>) const
    {
        if (i < n) {
            x[i] = xt[i];
            xa[i] = xt[i];
        } else {
            const long long j = i - n;
            y[j] = yt[j];
            ya[j] = yt[j];
        }
    }
};

// mixed precision: the new reference point (x_T, y_T) after a check, and
// y - y_ref for the next primal step's product
struct EpiRefUpdate : EpiBase {
    static constexpr int NR = 0;
    const double *xt, *yt, *y;
    double *xref, *yref;
    float* dy32;
    int n;
    __device__ void elem(long long i, Acc<NR>) const
    {
        if (i < n) {
            xref[i] = xt[i];
        } else {
            const long long j = i - n;
            yref[j] = yt[j];
            dy32[j] = (float)(y[j] - yt[j]);
        }
    }
};

// mixed precision: reference point and products zero before the first check
struct EpiRefZero : EpiBase {
    static constexpr int NR = 0;
    double *xref, *atyref, *yref, *axref;
    float* dy32;
    int n;
    __device__ void elem(long long i, Acc<NR>) const
    {
        if (i < n) {
            xref[i] = 0.0;
            atyref[i] = 0.0;
        } else {
            const long long j = i - n;
            yref[j] = 0.0;
            axref[j] = 0.0;
            dy32[j] = 0.0f;
        }
    }
};

// start point x0 = proj_X(0), y0 = 0, anchors and T(z) set to the start
struct EpiStart : EpiBase {
    static constexpr int NR = 0;
    BoundVec lv, uv;
    double *x, *xa, *xt, *y, *ya, *yt;
    int n;
    __device__ void elem(long long i, Acc<NR>) const
    {
        if (i < n) {
            const double v = clampd(0.0, lv[i], uv[i]);
            x[i] = v; xa[i] = v; xt[i] = v;
        } else {
            const long long j = i - n;
            y[j] = 0.0; ya[j] = 0.0; yt[j] = 0.0;
        }
    }
};

// SplitMix64 output for counter i with seed 0 (Steele, Lea and Flood 2014),
// mapped to [-1, 1): the power-iteration start vector, with its squared norm
struct EpiPowerStart : EpiBase {
    static constexpr int NR = 1;
    double* v;
    __device__ void elem(long long i, Acc<NR> a) const
    {
        unsigned long long z = (static_cast<unsigned long long>(i) + 1ull) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        const double val = 2.0 * u - 1.0;
        v[i] = val;
        a[0] += val * val;
    }
    __device__ void finalize(const double* t) const { ctrl->pw_norm = sqrt(t[0]); }
};

// y = M x with ||y||_2 left in ctrl->pw_norm
struct EpiNorm : EpiBase {
    static constexpr int NR = 1;
    const double* x;
    double* y;
    __device__ double xval(int j) const { return x[j]; }
    __device__ void row(int i, double s, Acc<NR> a) const
    {
        y[i] = s;
        a[0] += s * s;
    }
    __device__ void finalize(const double* t) const { ctrl->pw_norm = sqrt(t[0]); }
};

// v <- v / ctrl->pw_norm
struct EpiScale : EpiBase {
    static constexpr int NR = 0;
    double* v;
    double inv;
    __device__ void init() { inv = 1.0 / ctrl->pw_norm; }
    __device__ void elem(long long i, Acc<NR>) const { v[i] *= inv; }
};

struct EpiPlain : EpiBase {
    static constexpr int NR = 0;
    const double* x;
    double* y;
    __device__ double xval(int j) const { return x[j]; }
    __device__ void row(int i, double s, Acc<NR>) const { y[i] = s; }
};

struct EpiDot : EpiBase {
    static constexpr int NR = 1;
    const double *a, *b;
    __device__ void elem(long long i, Acc<NR> acc) const { acc[0] += a[i] * b[i]; }
    __device__ void finalize(const double* t) const { ctrl->pw_norm = t[0]; }
};

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int vec_grid(long long len)
{
    long long g = (len + TPB - 1) / TPB;
    if (g < 1) g = 1;
    if (g > VEC_GRID_MAX) g = VEC_GRID_MAX;
    return (int)g;
}

template <class E>
// the FP32 form only in a mixed-precision solve (a matrix keeps its FP32
// copy after one; an FP64 solve then still runs the FP64-only kernel)
static void launch_spmv_main(const CsrDev& M, const E& e, double* partials, bool mixed, hipStream_t s)
{
    if constexpr (E::BULK) {
        if (M.val32 && mixed) {
            k_spmv<E, true><<<M.nblk, TPB, 0, s>>>(M, e, partials);
            return;
        }
    }
    k_spmv<E, false><<<M.nblk, TPB, 0, s>>>(M, e, partials);
}

// blocks whose partials a product leaves for its finishing step
static int spmv_partial_blocks(const CsrDev& M) { return M.nparts > 1 ? vec_grid(M.rows) : M.nblk; }

// Product with epilogue e.  defer: leave e's partials in S.partials2 and
// launch no finishing kernel (the caller hands e to the next product's
// finishing kernel as `pre`; only valid when the product has no long rows
// to complete).  pre / pre_nblk: an earlier deferred epilogue finished first.
// leave_long: the long rows are completed by the next kernel (no finishing
// kernel at all when nothing reads this launch's reductions)
template <class E, class Pre = NoPre>
static hipError_t run_spmv(const DevState& S, const CsrDev& M, const E& e, hipStream_t s, bool defer = false,
                           const Pre& pre = Pre{}, int pre_nblk = 0, bool leave_long = false)
{
    double* part = defer ? S.partials2 : S.partials;
    // e.reduce == 0: no finishing step, except the completion of long rows
    const bool fin = e.reduce && E::NR > 0 && !defer;
    if (M.nparts > 1) {
        const int grid = vec_grid(M.rows);
        if (S.tev) (void)hipEventRecord(S.tev[0], s);
        launch_spmv_main(M, e, part, S.mixed != 0, s);
        k_rows<E><<<grid, TPB, 0, s>>>(M, e, part);
        if (S.tev) (void)hipEventRecord(S.tev[1], s);
        if (fin) k_vec_fin<E, Pre><<<1, FIN_T, 0, s>>>(grid, e, part, pre, pre_nblk, S.partials2);
        return hipGetLastError();
    }
    if (S.tev) (void)hipEventRecord(S.tev[0], s);
    launch_spmv_main(M, e, part, S.mixed != 0, s);
    if (S.tev) (void)hipEventRecord(S.tev[1], s);
    if (fin || (M.nlr > 0 && !defer && !leave_long))
        k_spmv_fin<E, Pre><<<1, FIN_T, 0, s>>>(M, e, part, pre, pre_nblk, S.partials2);
    return hipGetLastError();
}

template <class E>
static hipError_t run_vec(const DevState& S, long long len, const E& e, hipStream_t s, bool defer = false)
{
    const int grid = vec_grid(len);
    double* part = defer ? S.partials2 : S.partials;
    if (S.tev) (void)hipEventRecord(S.tev[0], s);
    k_vec<E><<<grid, TPB, 0, s>>>(len, e, part);
    if (S.tev) (void)hipEventRecord(S.tev[1], s);
    if (E::NR > 0 && !defer) k_vec_fin<E><<<1, FIN_T, 0, s>>>(grid, e, part);
    return hipGetLastError();
}

hipError_t launch_init_start(const DevState& S, hipStream_t s)
{
    EpiStart e{};
    e.ctrl = S.ctrl;
    e.lv = S.lv; e.uv = S.uv;
    e.x = S.x; e.xa = S.xa; e.xt = S.xt; e.y = S.y; e.ya = S.ya; e.yt = S.yt;
    e.n = S.n;
    return run_vec(S, (long long)S.n + S.m, e, s);
}

static HalpernX halpern_x(const DevState& S, int store_delta)
{
    HalpernX h{};
    h.xa = S.xa; h.c = S.c; h.lv = S.lv; h.uv = S.uv; h.x = S.x; h.d = S.dx;
    h.store = store_delta;
    return h;
}

static EpiProx prox_epi(const DevState& S, int store_delta)
{
    EpiProx e{};
    e.ctrl = S.ctrl;
    e.y = S.y; e.x = S.x; e.c = S.c; e.qd = S.qd; e.lv = S.lv; e.uv = S.uv; e.xt = S.xt;
    e.xbar = S.xbar;
    e.hx = halpern_x(S, store_delta);
    if (S.mixed) { e.dy32 = S.dy32; e.atyref = S.atyref; e.xref = S.xref; e.dxb32 = S.dxb32; }
    return e;
}

// The primal step's finishing work (the movement of x and, before a check,
// the unboundedness pieces, and the inner tolerance) feeds nothing the dual
// step reads, so it is carried into the dual step's finishing kernel when
// the product has no long rows to complete there.
bool prox_diag_deferrable(const DevState& S) { return S.AT.nlr == 0; }

static EpiDual dual_epi(const DevState& S, int store_delta, long long tk, long long kk);

hipError_t launch_prox_diag(const DevState& S, int store_delta, long long tk, bool reduce, long long lr_k,
                            long long lr_t, hipStream_t s)
{
    EpiProx e = prox_epi(S, store_delta);
    e.hx.tk = tk;
    e.reduce = reduce ? 1 : 0;
    if (lr_k >= 0) {
        if (!S.ylr || S.A.nlr == 0) return hipErrorInvalidValue;
        e.lrd = dual_epi(S, 0, lr_t, lr_k);
        e.lrd.reduce = 0;
        e.lrd.ylr_out = S.ylr + (size_t)((lr_k + 1) & 1) * S.A.nlr;
        e.ylr_in = S.ylr + (size_t)(lr_k & 1) * S.A.nlr;
        e.lr_info = S.A.lr_info;
        e.lr_seg = S.A.seg_part;
        e.lr_n = S.A.nlr;
        e.lr_coop = S.A.nlr_coop;
        for (int j = 0; j < 3; ++j) e.lr0[j] = S.A.lr0[j];
    }
    return run_spmv(S, S.AT, e, s, prox_diag_deferrable(S));
}

hipError_t launch_rhs(const DevState& S, hipStream_t s)
{
    EpiRhs e{};
    e.ctrl = S.ctrl;
    e.y = S.y; e.x = S.x; e.c = S.c; e.rhs = S.rhs;
    if (S.mixed) { e.dy32 = S.dy32; e.atyref = S.atyref; }
    return run_spmv(S, S.AT, e, s);
}

static EpiXbar xbar_epi(const DevState& S, int store_delta);

hipError_t launch_rhs_grad(const DevState& S, long long seq, bool pre_xbar, hipStream_t s)
{
    EpiRhsGrad e{};
    e.ctrl = S.ctrl;
    e.y = S.y; e.x = S.x; e.c = S.c; e.xt = S.xt; e.lv = S.lv; e.uv = S.uv; e.rhs = S.rhs; e.g = S.g;
    e.dstat = S.dstat; e.seq = seq;
    if (S.mixed) { e.dy32 = S.dy32; e.atyref = S.atyref; }
    // the previous iteration's x_bar / Halpern finishing work (its inner
    // tolerance update first: this kernel's decision reads it)
    if (pre_xbar) return run_spmv(S, S.AT, e, s, false, xbar_epi(S, 0), vec_grid(S.n));
    return run_spmv(S, S.AT, e, s);
}

hipError_t launch_tail(const DevState& S, const double* v, double* tail, bool bulk, hipStream_t s)
{
    if (S.R.rows == 0) return hipSuccess;
    if (bulk) {
        EpiTail<true> e{};
        e.ctrl = S.ctrl;
        e.v = v; e.tail = tail;
        return run_spmv(S, S.R, e, s);
    }
    EpiTail<false> e{};
    e.ctrl = S.ctrl;
    e.v = v; e.tail = tail;
    return run_spmv(S, S.R, e, s);
}

hipError_t launch_ginit(const DevState& S, long long seq, hipStream_t s)
{
    if (S.R.rows) {
        hipError_t err = launch_tail(S, S.xt, S.xt + S.n, false, s);
        if (err != hipSuccess) return err;
    }
    EpiGinit e{};
    e.ctrl = S.ctrl;
    e.xt = S.xt; e.rhs = S.rhs; e.lv = S.lv; e.uv = S.uv; e.g = S.g;
    e.dstat = S.dstat; e.seq = seq;
    return run_spmv(S, S.Q, e, s);
}

// The inner step's kernels are compiled per storage mode of the box (one
// pair, byte classes, arrays; BoundVec): the host picks the instance.
template <int BM>
static hipError_t launch_dir_m(const DevState& S, hipStream_t s)
{
    EpiDir<BM> e{};
    e.ctrl = S.ctrl;
    e.xt = S.xt; e.g = S.g; e.lv = S.lv; e.uv = S.uv; e.p = S.p;
    return run_vec(S, S.n, e, s);
}

template <int BM>
static hipError_t launch_hp_m(const DevState& S, hipStream_t s)
{
    EpiStepA<BM> e{};
    e.ctrl = S.ctrl;
    e.p = S.p; e.lv = S.lv; e.uv = S.uv; e.rhs = S.rhs; e.xt = S.xt; e.g = S.g; e.hp = S.hp;
    e.dstat = S.dstat; e.mixed = S.mixed;
    return run_spmv(S, S.Q, e, s);
}

template <int BM>
static hipError_t launch_update_m(const DevState& S, hipStream_t s)
{
    EpiStepB<BM> e{};
    e.ctrl = S.ctrl;
    e.p = S.p; e.hp = S.hp; e.lv = S.lv; e.uv = S.uv; e.xt = S.xt; e.g = S.g;
    e.dstat = S.dstat;
    return run_vec(S, S.n, e, s);
}

hipError_t launch_dir(const DevState& S, hipStream_t s)
{
    switch (S.lv.mode) {
    case 1: return launch_dir_m<1>(S, s);
    case 2: return launch_dir_m<2>(S, s);
    default: return launch_dir_m<0>(S, s);
    }
}

hipError_t launch_hp(const DevState& S, hipStream_t s)
{
    if (S.R.rows) {
        EpiTailHp t{};
        t.ctrl = S.ctrl;
        t.p = S.p; t.xt = S.xt; t.ptail = S.p + S.n; t.xtail = S.xt + S.n; t.mixed = S.mixed;
        hipError_t err = run_spmv(S, S.R, t, s);
        if (err != hipSuccess) return err;
    }
    switch (S.lv.mode) {
    case 1: return launch_hp_m<1>(S, s);
    case 2: return launch_hp_m<2>(S, s);
    default: return launch_hp_m<0>(S, s);
    }
}

hipError_t launch_update(const DevState& S, hipStream_t s)
{
    switch (S.lv.mode) {
    case 1: return launch_update_m<1>(S, s);
    case 2: return launch_update_m<2>(S, s);
    default: return launch_update_m<0>(S, s);
    }
}

static EpiXbar xbar_epi(const DevState& S, int store_delta)
{
    EpiXbar e{};
    e.ctrl = S.ctrl;
    e.xt = S.xt; e.xbar = S.xbar;
    e.hx = halpern_x(S, store_delta);
    if (S.mixed) { e.xref = S.xref; e.dxb32 = S.dxb32; }
    return e;
}

// x_bar and the Halpern average of x after an inner solve; its finishing
// work is carried into the dual step's finishing kernel (as for the
// closed-form primal step)
hipError_t launch_xbar(const DevState& S, int store_delta, long long tk, hipStream_t s)
{
    EpiXbar e = xbar_epi(S, store_delta);
    e.hx.tk = tk;
    return run_vec(S, S.n, e, s, true);
}

hipError_t launch_clip(const DevState& S, double* x, hipStream_t s)
{
    EpiClip e{};
    e.ctrl = S.ctrl;
    e.lv = S.lv; e.uv = S.uv; e.x = x;
    return run_vec(S, S.n, e, s);
}

static EpiDual dual_epi(const DevState& S, int store_delta, long long tk, long long kk)
{
    EpiDual e{};
    e.ctrl = S.ctrl;
    e.xbar = S.xbar; e.ya = S.ya; e.lc = S.lc; e.uc = S.uc;
    e.y = S.y; e.yt = S.yt; e.ytil = S.ytil; e.store = store_delta;
    e.tk = tk;
    e.kk = kk;
    if (S.mixed) { e.dxb32 = S.dxb32; e.axref = S.axref; e.yref = S.yref; e.dy32 = S.dy32; }
    return e;
}

hipError_t launch_dual(const DevState& S, int store_delta, int pre, long long tk, long long kk, bool reduce,
                       bool leave_long, hipStream_t s)
{
    EpiDual e = dual_epi(S, store_delta, tk, kk);
    e.reduce = reduce ? 1 : 0;
    // the long rows' copy for a later step that leaves them (closed-form path)
    if (S.ylr && kk >= 0) e.ylr_out = S.ylr + (size_t)((kk + 1) & 1) * S.A.nlr;
    if (leave_long && (reduce || store_delta || pre != PRE_PROX || !S.ylr || kk < 0)) return hipErrorInvalidValue;
    if (pre == PRE_PROX) {
        EpiProx pe = prox_epi(S, store_delta);
        pe.hx.tk = tk;
        return run_spmv(S, S.A, e, s, false, pe, spmv_partial_blocks(S.AT), leave_long);
    }
    if (pre == PRE_XBAR) {
        EpiXbar xe = xbar_epi(S, store_delta);
        xe.hx.tk = tk;
        return run_spmv(S, S.A, e, s, false, xe, vec_grid(S.n));
    }
    return run_spmv(S, S.A, e, s);
}

hipError_t launch_check(const DevState& S, const double* x, const double* y, int full, int dinf,
                        hipStream_t s)
{
    hipError_t err;
    if (full) {
        // certificate pieces first: the decision is taken in the last kernel
        EpiPinf ep{};
        ep.ctrl = S.ctrl;
        ep.ytil = S.ytil; ep.lv = S.lv; ep.uv = S.uv;
        if ((err = run_spmv(S, S.AT, ep, s)) != hipSuccess) return err;
        if (dinf) {
            if ((err = launch_tail(S, S.dx, S.dx + S.n, false, s)) != hipSuccess) return err;
            EpiAd ea{};
            ea.ctrl = S.ctrl;
            ea.d = S.dx; ea.lc = S.lc; ea.uc = S.uc;
            if ((err = run_spmv(S, S.A, ea, s)) != hipSuccess) return err;
            EpiQd eqd{};
            eqd.ctrl = S.ctrl;
            eqd.d = S.dx;
            if ((err = run_spmv(S, S.Q, eqd, s)) != hipSuccess) return err;
        }
    }
    EpiAty et{};
    et.ctrl = S.ctrl;
    et.y = y; et.aty = S.aty;
    if (full && S.mixed) et.atyref = S.atyref;
    if ((err = run_spmv(S, S.AT, et, s)) != hipSuccess) return err;
    EpiAx ex{};
    ex.ctrl = S.ctrl;
    ex.x = x; ex.y = y; ex.ya = full ? S.ya : nullptr; ex.lc = S.lc; ex.uc = S.uc;
    if (full && S.mixed) ex.axref = S.axref;
    if ((err = run_spmv(S, S.A, ex, s)) != hipSuccess) return err;
    if (S.R.rows) {
        // the operand needs room for its tail: x_T has it, any other x is copied
        double* xq = S.xt;
        if (x != S.xt) {
            xq = S.v1;
            if ((err = hipMemcpyAsync(xq, x, sizeof(double) * S.n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
                return err;
        }
        if ((err = launch_tail(S, xq, xq + S.n, false, s)) != hipSuccess) return err;
        x = xq;
    }
    EpiQx eq{};
    eq.ctrl = S.ctrl;
    eq.x = x; eq.xa = full ? S.xa : nullptr; eq.c = S.c; eq.aty = S.aty; eq.lv = S.lv; eq.uv = S.uv;
    eq.dcheck = S.dcheck; eq.full = full;
    return run_spmv(S, S.Q, eq, s);
}

hipError_t launch_restart_copy(const DevState& S, hipStream_t s)
{
    EpiRestart e{};
    e.ctrl = S.ctrl;
    e.xt = S.xt; e.yt = S.yt; e.x = S.x; e.xa = S.xa; e.y = S.y; e.ya = S.ya; e.n = S.n;
    return run_vec(S, (long long)S.n + S.m, e, s);
}

hipError_t launch_ref_update(const DevState& S, hipStream_t s)
{
    if (!S.mixed) return hipSuccess;
    EpiRefUpdate e{};
    e.ctrl = S.ctrl;
    e.xt = S.xt; e.yt = S.yt; e.y = S.y; e.xref = S.xref; e.yref = S.yref; e.dy32 = S.dy32; e.n = S.n;
    return run_vec(S, (long long)S.n + S.m, e, s);
}

hipError_t launch_ref_zero(const DevState& S, hipStream_t s)
{
    if (!S.mixed) return hipSuccess;
    EpiRefZero e{};
    e.ctrl = S.ctrl;
    e.xref = S.xref; e.atyref = S.atyref; e.yref = S.yref; e.axref = S.axref; e.dy32 = S.dy32; e.n = S.n;
    return run_vec(S, (long long)S.n + S.m, e, s);
}

hipError_t launch_power_start(const DevState& S, double* v, int len, hipStream_t s)
{
    EpiPowerStart e{};
    e.ctrl = S.ctrl;
    e.v = v;
    return run_vec(S, len, e, s);
}

hipError_t launch_spmv_norm(const DevState& S, const CsrDev& M, const double* x, double* y,
                            hipStream_t s)
{
    EpiNorm e{};
    e.ctrl = S.ctrl;
    e.x = x; e.y = y;
    return run_spmv(S, M, e, s);
}

hipError_t launch_scale(const DevState& S, double* v, int len, hipStream_t s)
{
    EpiScale e{};
    e.ctrl = S.ctrl;
    e.v = v;
    return run_vec(S, len, e, s);
}

hipError_t launch_spmv_plain(const DevState& S, const CsrDev& M, const double* x, double* y,
                             hipStream_t s)
{
    EpiPlain e{};
    e.ctrl = S.ctrl;
    e.x = x; e.y = y;
    return run_spmv(S, M, e, s);
}

__global__ __launch_bounds__(TPB) void k_to_f32(long long len, const double* src, float* dst)
{
    const long long stride = (long long)gridDim.x * TPB;
    for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < len; i += stride) dst[i] = (float)src[i];
}

hipError_t launch_to_f32(const double* src, float* dst, long long len, hipStream_t s)
{
    if (len > 0) k_to_f32<<<vec_grid(len), TPB, 0, s>>>(len, src, dst);
    return hipGetLastError();
}

hipError_t launch_dot(const DevState& S, const double* a, const double* b, int len, hipStream_t s)
{
    EpiDot e{};
    e.ctrl = S.ctrl;
    e.a = a; e.b = b;
    return run_vec(S, len, e, s);
}

}  // namespace pdhcg
