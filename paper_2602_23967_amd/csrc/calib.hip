// calib.hip -- a measurement utility, not part of the method: the rate at
// which the device serves random 8-byte gathers from a vector of n doubles
// when the gathering blocks keep to the same XCD-keyed column parts as the
// column-partitioned products (block b reads part (b mod 8) mod 4).  The
// large products' inner loop is bound by this rate rather than by HBM
// bytes, so the bench reports the product's gather rate against it.
#include <hip/hip_runtime.h>

#include <chrono>
#include <string>

#include "host_internal.h"
#include "pdhcg_internal.h"

namespace pdhcg {
namespace {

constexpr int CAL_T = 256;
constexpr int CAL_PER = 8;

__device__ __forceinline__ unsigned mix32(unsigned a)
{
    a ^= a >> 16;
    a *= 0x7feb352dU;
    a ^= a >> 15;
    a *= 0x846ca68bU;
    a ^= a >> 16;
    return a;
}

// every thread sums CAL_PER pseudo-random entries of its block's part
__global__ __launch_bounds__(CAL_T) void k_gather_calib(const double* __restrict__ x, long long part_len,
                                                        int parts, double* __restrict__ out)
{
    const int part = (int)(blockIdx.x & 7u) % parts;
    const unsigned t = blockIdx.x * CAL_T + threadIdx.x;
    const double* xp = x + (long long)part * part_len;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < CAL_PER; ++i) s += xp[mix32(t * CAL_PER + i) % (unsigned)part_len];
    out[t] = s;
}

}  // namespace
}  // namespace pdhcg

extern "C" int qp_measure_gather_rate(int64_t n, int64_t gathers, int32_t repeats, double* gathers_per_s)
{
    using namespace pdhcg;
    if (n < (int64_t)NPARTS || n > (int64_t)1 << 31 || gathers < CAL_T * CAL_PER || repeats < 1 || !gathers_per_s)
        return fail(QP_ERR_INVALID_ARG, "need n >= 4 (< 2^31), gathers >= 2048, repeats >= 1, an output");
    const long long blocks = (gathers + CAL_T * CAL_PER - 1) / (CAL_T * CAL_PER);
    if (blocks > (1ll << 22)) return fail(QP_ERR_INVALID_ARG, "too many gathers");   // thread ids fit 32 bits
    const long long part_len = n / NPARTS;
    // a stream of its own, never the legacy null stream: once the null
    // stream has run kernels, a request server created later in the same
    // process measured its batched launches up to 5x slower beside its
    // single-problem workers
    double *x = nullptr, *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        if (s) (void)hipStreamSynchronize(s);
        if (x) (void)hipFree(x);
        if (out) (void)hipFree(out);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (s) (void)hipStreamDestroy(s);
    };
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&x, sizeof(double) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&out, sizeof(double) * (size_t)blocks * CAL_T);
    if (e == hipSuccess) e = hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        cleanup();
        return fail(QP_ERR_DEVICE, std::string("gather calibration: ") + hipGetErrorString(e));
    }
    float ms = 0.0f;
    for (int w = 0; w < 3 && e == hipSuccess; ++w) {
        k_gather_calib<<<(unsigned)blocks, CAL_T, 0, s>>>(x, part_len, NPARTS, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    for (int r = 0; r < repeats && e == hipSuccess; ++r) {
        k_gather_calib<<<(unsigned)blocks, CAL_T, 0, s>>>(x, part_len, NPARTS, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    cleanup();
    if (e != hipSuccess) return fail(QP_ERR_DEVICE, std::string("gather calibration: ") + hipGetErrorString(e));
    *gathers_per_s = ms > 0.0f ? (double)blocks * CAL_T * CAL_PER * repeats / (ms * 1e-3) : 0.0;
    return 0;
}
