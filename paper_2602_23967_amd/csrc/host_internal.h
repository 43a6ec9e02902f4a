// Host-side helpers shared by the single-problem / batched API (host.cpp)
// and the request server (serve.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pdhcg.h"
#include "prep.h"

namespace pdhcg {

// A region of device memory the library does not own (the static workspace of
// qp_batch_solve_static): allocations are carved from it in 256-byte steps
// and never freed; one that does not fit fails with QP_ERR_INVALID_ARG.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
};

// qp_batch_create on a stream lent by the caller (NULL: the batch makes its
// own).  With an arena, every device buffer of the batch comes from it, the
// batch uses `lane` as given (NULL is the null stream) and creates no stream
// or event: nothing is allocated on the device.
int batch_create(hipStream_t lane, int64_t count, const int64_t* var_off, const int64_t* row_off,
                 const int64_t* Qp, const int32_t* Qj, const double* Qv,
                 const int64_t* Ap, const int32_t* Aj, const double* Av,
                 const double* c, const double* b, const char* sense,
                 const double* lb, const double* ub, qp_batch** out, Arena* arena = nullptr);

// asynchronous batched solve: launch on the batch's stream, poll
// (1 finished, 0 running, < 0 error), finish (fetches the outcomes and
// returns the number of OPTIMAL instances)
int batch_launch(qp_batch* bt, const qp_params* params);
int batch_poll(qp_batch* bt);
int batch_finish(qp_batch* bt);
// after batch_finish: outcome of instance i
void batch_info(const qp_batch* bt, int64_t i, qp_info* info);
// after batch_finish: the returned x and y of every instance in one copy each
// (packed like the problem; certificates in place of the iterates, scaled as
// in qp_batch_result)
int batch_results_all(qp_batch* bt, std::vector<double>& x, std::vector<double>& y);

}  // namespace pdhcg
