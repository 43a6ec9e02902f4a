// device_math.h -- elementwise pieces of the method shared by the gfx950
// kernels (kernels.hip, batch.hip): projections onto the sets of Section 2,
// terms of the support function p, the gradient split of the box-QP solver,
// and NaN-propagating reduction operators.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace pdhcg {

enum { R_SUM = 0, R_MAX = 1, R_MIN = 2 };

__device__ __forceinline__ double rcomb(int kind, double a, double b)
{
    if (kind == R_SUM) return a + b;
    if (a != a) return a;
    if (b != b) return b;
    if (kind == R_MAX) return a > b ? a : b;
    return a < b ? a : b;
}

// identities: every MAX slot reduces magnitudes, so 0 is its identity
__device__ __forceinline__ double rid(int kind) { return kind == R_MIN ? INFINITY : 0.0; }

// status word in pinned host memory: a single 64-bit store (no fence; the
// host only needs it eventually, and the kernel's end publishes it anyway)
__device__ __forceinline__ void post_status(unsigned long long* w, long long seq, int flag)
{
    __hip_atomic_store(w, (static_cast<unsigned long long>(seq) << 1) | (flag ? 1ull : 0ull),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ double clampd(double v, double l, double u)
{
    return v < l ? l : (v > u ? u : v);
}

// sign set Y_i of a row (Section 2): {0} free, R+ upper only, R- lower only, R both
__device__ __forceinline__ double projY(double v, double l, double u)
{
    const bool lf = isfinite(l), uf = isfinite(u);
    if (lf && uf) return v;
    if (uf) return v > 0.0 ? v : 0.0;
    if (lf) return v < 0.0 ? v : 0.0;
    return 0.0;
}

// sign set R_i of a variable (Section 2): {0} free, R- upper only, R+ lower only, R both
__device__ __forceinline__ double projR(double v, double l, double u)
{
    const bool lf = isfinite(l), uf = isfinite(u);
    if (lf && uf) return v;
    if (uf) return v < 0.0 ? v : 0.0;
    if (lf) return v > 0.0 ? v : 0.0;
    return 0.0;
}

// recession cone of [l, u]: {0} bounded, R+ lower only, R- upper only, R free
__device__ __forceinline__ double projRec(double v, double l, double u)
{
    const bool lf = isfinite(l), uf = isfinite(u);
    if (lf && uf) return 0.0;
    if (lf) return v > 0.0 ? v : 0.0;
    if (uf) return v < 0.0 ? v : 0.0;
    return v;
}

// terms of p(z; l, u) = u'z+ - l'z- (0 * inf = 0) and of its magnitude
__device__ __forceinline__ double supp(double z, double l, double u)
{
    return z > 0.0 ? u * z : (z < 0.0 ? l * z : 0.0);
}
__device__ __forceinline__ double supp_abs(double z, double l, double u)
{
    return z > 0.0 ? fabs(u) * z : (z < 0.0 ? -fabs(l) * z : 0.0);
}

// Gradient split at a feasible x for the box QP (free gradient phi, chopped
// gradient beta, reduced free gradient phit for step abar).
struct Split {
    double phi, beta, phit;
};

__device__ __forceinline__ Split split(double x, double g, double l, double u, double abar)
{
    Split s{0.0, 0.0, 0.0};
    if (x > l && x < u) {
        s.phi = g;
        if (g > 0.0) s.phit = isfinite(l) ? fmin((x - l) / abar, g) : g;
        else if (g < 0.0) s.phit = isfinite(u) ? fmax((x - u) / abar, g) : g;
    } else if (l < u) {
        if (x <= l) s.beta = g < 0.0 ? g : 0.0;
        else s.beta = g > 0.0 ? g : 0.0;
    }
    return s;
}


}  // namespace pdhcg
