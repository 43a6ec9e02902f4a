// prep.cpp -- host-only preparation of a problem: input validation, the
// transpose, the SpMV work schedules and the storage class of the box.  No
// device code and no HIP calls: besides the library build it compiles with a
// plain C++ compiler (the sanitizer builds of the tests).
#include "prep.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>

namespace pdhcg {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// validation (host only, runs before any device call)
// ---------------------------------------------------------------------------

int check_csr(const char* name, int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj,
              const double* v)
{
    if (!rp) return fail(QP_ERR_INVALID_ARG, std::string(name) + ": row pointer is NULL");
    if (rp[0] != 0) return fail(QP_ERR_INVALID_ARG, std::string(name) + ": rowptr[0] != 0");
    for (int64_t i = 0; i < rows; ++i)
        if (rp[i + 1] < rp[i])
            return fail(QP_ERR_INVALID_ARG, std::string(name) + ": row pointers decrease at row " +
                                                std::to_string(i));
    const int64_t nnz = rp[rows];
    if (nnz >= (int64_t)INT32_MAX)
        return fail(QP_ERR_INVALID_ARG, std::string(name) + ": nnz must be below 2^31");
    if (nnz > 0 && (!cj || !v))
        return fail(QP_ERR_INVALID_ARG, std::string(name) + ": column or value array is NULL");
    for (int64_t i = 0; i < rows; ++i) {
        int64_t prev = -1;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = cj[k];
            if (j < 0 || j >= cols)
                return fail(QP_ERR_INVALID_ARG, std::string(name) + ": column out of range in row " +
                                                    std::to_string(i));
            if (j <= prev)
                return fail(QP_ERR_INVALID_ARG, std::string(name) +
                                                    ": columns not sorted or duplicated in row " +
                                                    std::to_string(i));
            if (!std::isfinite(v[k]))
                return fail(QP_ERR_INVALID_ARG, std::string(name) + ": non-finite value in row " +
                                                    std::to_string(i));
            prev = j;
        }
    }
    return 0;
}

// transpose of an (rows x cols) CSR by counting sort (columns stay sorted)
void transpose(int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj, const double* v,
               std::vector<int64_t>& tp, std::vector<int32_t>& tj, std::vector<double>& tv)
{
    const int64_t nnz = rp[rows];
    tp.assign(cols + 1, 0);
    tj.resize(nnz);
    tv.resize(nnz);
    for (int64_t k = 0; k < nnz; ++k) tp[cj[k] + 1]++;
    for (int64_t j = 0; j < cols; ++j) tp[j + 1] += tp[j];
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t d = fill[cj[k]]++;
            tj[d] = (int32_t)i;
            tv[d] = v[k];
        }
}

int check_symmetric(int64_t n, const int64_t* rp, const int32_t* cj, const double* v)
{
    std::vector<int64_t> tp;
    std::vector<int32_t> tj;
    std::vector<double> tv;
    transpose(n, n, rp, cj, v, tp, tj, tv);
    for (int64_t i = 0; i <= n; ++i)
        if (tp[i] != rp[i]) return fail(QP_ERR_NOT_SYMMETRIC, "Q: sparsity pattern is not symmetric");
    for (int64_t k = 0; k < rp[n]; ++k) {
        if (tj[k] != cj[k]) return fail(QP_ERR_NOT_SYMMETRIC, "Q: sparsity pattern is not symmetric");
        const double a = v[k], b = tv[k];
        if (std::fabs(a - b) > 1e-14 * std::max(std::fabs(a), std::fabs(b)))
            return fail(QP_ERR_NOT_SYMMETRIC, "Q: values are not symmetric");
    }
    return 0;
}

int check_vec(const char* name, int64_t len, const double* v, bool allow_inf)
{
    if (!v) return fail(QP_ERR_INVALID_ARG, std::string(name) + " is NULL");
    for (int64_t i = 0; i < len; ++i) {
        if (std::isnan(v[i]) || (!allow_inf && !std::isfinite(v[i])))
            return fail(QP_ERR_INVALID_ARG, std::string(name) + ": invalid entry " + std::to_string(i));
    }
    return 0;
}

int check_bounds(const char* name, int64_t len, const double* l, const double* u)
{
    for (int64_t i = 0; i < len; ++i) {
        if (std::isnan(l[i]) || std::isnan(u[i]) || l[i] > u[i] || l[i] == INFINITY || u[i] == -INFINITY)
            return fail(QP_ERR_INVALID_ARG, std::string(name) + ": invalid bounds at " + std::to_string(i));
    }
    return 0;
}


// ---------------------------------------------------------------------------
// SpMV schedule: greedy row blocks of <= NNZ_CAP nonzeros and <= ROWS_CAP
// rows; a row longer than NNZ_CAP is an item of its own when it has at most
// ROW_PASS_CAP nonzeros, else NNZ_CAP-sized segments
// ---------------------------------------------------------------------------

void build_plan(int64_t rows, const int64_t* rp, std::vector<BlkDesc>& blk, int& nlr, int& nseg_tot)
{
    blk.clear();
    nlr = 0;
    nseg_tot = 0;
    int64_t r = 0;
    while (r < rows) {
        const int64_t L = rp[r + 1] - rp[r];
        if (L > NNZ_CAP && L <= ROW_PASS_CAP) {
            blk.push_back({(int)r, 1, (int)rp[r], (int)rp[r + 1], 0, 0, 0, 0});
            ++r;
            continue;
        }
        if (L > NNZ_CAP) {
            const int nseg = (int)((L + NNZ_CAP - 1) / NNZ_CAP);
            for (int s = 0; s < nseg; ++s) {
                const int64_t a = rp[r] + (int64_t)s * NNZ_CAP;
                const int64_t b = std::min(a + (int64_t)NNZ_CAP, rp[r + 1]);
                blk.push_back({(int)r, 0, (int)a, (int)b, nlr, s, nseg, nseg_tot});
            }
            ++nlr;
            nseg_tot += nseg;
            ++r;
            continue;
        }
        const int64_t start = r;
        int64_t nnz = 0;
        while (r < rows && r - start < ROWS_CAP) {
            const int64_t Lr = rp[r + 1] - rp[r];
            if (Lr > NNZ_CAP || nnz + Lr > NNZ_CAP) break;
            nnz += Lr;
            ++r;
        }
        blk.push_back({(int)start, (int)(r - start), (int)rp[start], (int)rp[r], 0, 0, 0, 0});
    }
    if (blk.empty()) blk.push_back({0, 0, 0, 0, 0, 0, 0, 0});
}

// Column-partitioned layout (see pdhcg_internal.h): part p holds the entries
// of columns [p*w, (p+1)*w), w = ceil(cols / NPARTS), stored part after part
// with absolute row pointers; each part gets row blocks of <= NNZ_CAP
// nonzeros and <= PART_ROWS_CAP rows, and the blocks are interleaved so that
// block b belongs to part b % NPARTS.  Returns false (no partitioning) when a
// row of a part exceeds NNZ_CAP.
bool build_parts(int64_t rows, int64_t cols, const int64_t* rp, const int32_t* cj, const double* v,
                 std::vector<int>& prow, std::vector<int32_t>& pcol, std::vector<double>& pval,
                 std::vector<BlkDesc>& blk)
{
    const int64_t w = (cols + NPARTS - 1) / NPARTS;
    const int64_t nnz = rp[rows];
    // per (row, part) counts
    std::vector<int64_t> cnt((size_t)NPARTS * rows, 0);
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) cnt[(size_t)(cj[k] / w) * rows + i]++;
    for (size_t q = 0; q < cnt.size(); ++q)
        if (cnt[q] > NNZ_CAP) return false;
    prow.assign((size_t)NPARTS * (rows + 1), 0);
    int64_t off = 0;
    for (int p = 0; p < NPARTS; ++p) {
        int* pr = prow.data() + (size_t)p * (rows + 1);
        pr[0] = (int)off;
        for (int64_t i = 0; i < rows; ++i) {
            off += cnt[(size_t)p * rows + i];
            pr[i + 1] = (int)off;
        }
    }
    pcol.resize(nnz);
    pval.resize(nnz);
    std::vector<int64_t> fill(NPARTS);
    for (int64_t i = 0; i < rows; ++i) {
        for (int p = 0; p < NPARTS; ++p) fill[p] = prow[(size_t)p * (rows + 1) + i];
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int p = (int)(cj[k] / w);
            pcol[fill[p]] = cj[k];
            pval[fill[p]] = v[k];
            ++fill[p];
        }
    }
    std::vector<std::vector<BlkDesc>> per(NPARTS);
    size_t nb = 0;
    for (int p = 0; p < NPARTS; ++p) {
        const int* pr = prow.data() + (size_t)p * (rows + 1);
        int64_t r = 0;
        while (r < rows) {
            const int64_t start = r;
            int64_t z = 0;
            while (r < rows && r - start < PART_ROWS_CAP) {
                const int64_t L = pr[r + 1] - pr[r];
                if (z + L > NNZ_CAP) break;
                z += L;
                ++r;
            }
            per[p].push_back({(int)start, (int)(r - start), pr[start], pr[r], p, 0, 0, 0});
        }
        nb = std::max(nb, per[p].size());
    }
    blk.clear();
    for (size_t i = 0; i < nb; ++i)
        for (int p = 0; p < NPARTS; ++p)
            blk.push_back(i < per[p].size() ? per[p][i] : BlkDesc{0, 0, 0, 0, p, 0, 0, 0});
    return true;
}

// Storage of the variable bounds (BoundVec, pdhcg_internal.h): 1 when every
// variable has the same (l, u) pair, 2 when at most 256 distinct pairs occur
// (compared bit for bit, so every value is kept exactly; cls, tl, tu are
// filled), else 0 (the two arrays).  PDHCG_BOUND_STORAGE=arrays in the
// environment forces 0 (to check that every storage gives the same bits).
int classify_bounds(const std::vector<double>& lv, const std::vector<double>& uv, std::vector<unsigned char>& cls,
                    std::vector<double>& tl, std::vector<double>& tu)
{
    const size_t n = lv.size();
    const char* force = std::getenv("PDHCG_BOUND_STORAGE");
    if (n == 0 || (force && std::strcmp(force, "arrays") == 0)) return 0;
    typedef std::pair<uint64_t, uint64_t> Key;
    std::map<Key, int> index;
    std::vector<Key> keys;
    cls.assign(n, 0);
    int last = -1;
    Key lastkey{0, 0};
    for (size_t i = 0; i < n; ++i) {
        Key key;
        std::memcpy(&key.first, &lv[i], sizeof(double));
        std::memcpy(&key.second, &uv[i], sizeof(double));
        if (last < 0 || key != lastkey) {
            auto it = index.find(key);
            if (it != index.end()) {
                last = it->second;
            } else {
                if (keys.size() == 256) return 0;
                last = (int)keys.size();
                index.emplace(key, last);
                keys.push_back(key);
            }
            lastkey = key;
        }
        cls[i] = (unsigned char)last;
    }
    tl.resize(keys.size());
    tu.resize(keys.size());
    for (size_t c = 0; c < keys.size(); ++c) {
        std::memcpy(&tl[c], &keys[c].first, sizeof(double));
        std::memcpy(&tu[c], &keys[c].second, sizeof(double));
    }
    return keys.size() == 1 ? 1 : 2;
}

}  // namespace pdhcg
