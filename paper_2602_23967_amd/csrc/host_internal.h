// Host-side helpers shared by the single-problem / batched API (host.cpp)
// and the request server (serve.cpp). Not part of the public ABI.
#pragma once

#include <string>

#include "../../include/pdhcg.h"

namespace pdhcg {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);
double now_s();

// input validation shared by every entry point that takes a problem
int check_csr(const char* name, int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj,
              const double* v);
int check_symmetric(int64_t n, const int64_t* rp, const int32_t* cj, const double* v);
int check_vec(const char* name, int64_t len, const double* v, bool allow_inf);
int check_bounds(const char* name, int64_t len, const double* l, const double* u);

// asynchronous batched solve: launch on the batch's stream, poll
// (1 finished, 0 running, < 0 error), finish (fetches the outcomes and
// returns the number of OPTIMAL instances)
int batch_launch(qp_batch* bt, const qp_params* params);
int batch_poll(qp_batch* bt);
int batch_finish(qp_batch* bt);

}  // namespace pdhcg
