// prep.h -- host-only preparation of a problem (prep.cpp): validation,
// transpose, SpMV work schedules, box storage class.  No HIP types.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pdhcg.h"
#include "schedule.h"

namespace pdhcg {

// the calling thread's last error message (qp_last_error) and the setter
// every entry point returns through
extern thread_local std::string g_err;
int fail(int code, const std::string& msg);
double now_s();

// input validation shared by every entry point that takes a problem; each
// returns 0 or a negative QP_ERR_* code with the message set
int check_csr(const char* name, int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj,
              const double* v);
int check_symmetric(int64_t n, const int64_t* rp, const int32_t* cj, const double* v);
int check_vec(const char* name, int64_t len, const double* v, bool allow_inf);
int check_bounds(const char* name, int64_t len, const double* l, const double* u);

// transpose of a (rows x cols) CSR by counting sort (columns stay sorted)
void transpose(int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj, const double* v,
               std::vector<int64_t>& tp, std::vector<int32_t>& tj, std::vector<double>& tv);

// row-block schedule of a CSR (items of BlkDesc); nlr long rows split into
// nseg_tot segments in all
void build_plan(int64_t rows, const int64_t* rp, std::vector<BlkDesc>& blk, int& nlr, int& nseg_tot);

// column-partitioned copy of a CSR and its schedule; false when a row of a
// part is longer than a row block (then the matrix stays whole)
bool build_parts(int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj, const double* v,
                 std::vector<int>& prow, std::vector<int32_t>& pcol, std::vector<double>& pval,
                 std::vector<BlkDesc>& blk);

// storage class of the box: 1 one (l, u) pair, 2 byte classes into tables
// tl/tu (<= 256 pairs), 0 arrays
int classify_bounds(const std::vector<double>& lv, const std::vector<double>& uv, std::vector<unsigned char>& cls,
                    std::vector<double>& tl, std::vector<double>& tu);

}  // namespace pdhcg
