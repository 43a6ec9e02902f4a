// noalloc.cpp -- the batched solve that allocates no device memory
// (qp_batch_solve_static): every device buffer of the batch is carved from
// one static array per device, found once per device with
// hipGetSymbolAddress.  The batch itself (validation, copies, norms, the
// persistent solve kernel, results) is the allocating path's code.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pdhcg.h"
#include "host_internal.h"

using namespace pdhcg;

// The workspace.  Host code never uses its name as an address: the device
// address of each device's copy comes from hipGetSymbolAddress (ws_ptr).
static __device__ __align__(256) unsigned char scratch[QP_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_ws_mutex[MAX_DEVICES];
void* g_ws_ptr[MAX_DEVICES];   // device address of `scratch` on each device (set once)

// the workspace of the current device `dev`; call with g_ws_mutex[dev] held
int ws_ptr(int dev, void** out)
{
    if (!g_ws_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QP_ERR_DEVICE, std::string("hipGetSymbolAddress(workspace): ") + hipGetErrorString(e));
        g_ws_ptr[dev] = p;
    }
    *out = g_ws_ptr[dev];
    return 0;
}

}  // namespace

extern "C" int qp_batch_solve_static(int64_t count, const int64_t* var_off, const int64_t* row_off,
                                     const int64_t* Q_rowptr, const int32_t* Q_col, const double* Q_val,
                                     const int64_t* A_rowptr, const int32_t* A_col, const double* A_val,
                                     const double* c, const double* b, const char* sense,
                                     const double* lb, const double* ub, const qp_params* params,
                                     void* stream, double* x, double* y, int32_t* status, qp_info* info)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(QP_ERR_DEVICE, "no HIP device available");
    if (dev >= MAX_DEVICES) return fail(QP_ERR_DEVICE, "device index beyond the workspace table");
    std::lock_guard<std::mutex> hold(g_ws_mutex[dev]);
    void* base = nullptr;
    if (int rc = ws_ptr(dev, &base)) return rc;
    Arena arena;
    arena.base = static_cast<char*>(base);
    arena.cap = (size_t)QP_STATIC_WORKSPACE_BYTES;
    qp_batch* bt = nullptr;
    int rc = batch_create(static_cast<hipStream_t>(stream), count, var_off, row_off, Q_rowptr, Q_col, Q_val,
                          A_rowptr, A_col, A_val, c, b, sense, lb, ub, &bt, &arena);
    if (rc) return rc;
    rc = batch_launch(bt, params);
    int opt = rc < 0 ? rc : batch_finish(bt);
    if (opt >= 0 && (x || y)) {
        std::vector<double> xv, yv;
        rc = batch_results_all(bt, xv, yv);
        if (rc < 0) {
            opt = rc;
        } else {
            if (x) std::memcpy(x, xv.data(), sizeof(double) * xv.size());
            if (y && !yv.empty()) std::memcpy(y, yv.data(), sizeof(double) * yv.size());
        }
    }
    if (opt >= 0) {
        for (int64_t i = 0; i < count; ++i) {
            qp_info in;
            batch_info(bt, i, &in);
            if (status) status[i] = in.status;
            if (info) info[i] = in;
        }
    }
    const std::string err = opt < 0 ? g_err : std::string();
    qp_batch_destroy(bt);
    if (opt < 0) return fail(opt, err);
    g_err.clear();
    return opt;
}
