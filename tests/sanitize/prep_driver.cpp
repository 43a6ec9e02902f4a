// Drives the library's host-only preparation code (csrc/prep.cpp: input
// validation, transpose, SpMV work schedules, box storage class) on valid
// and malformed inputs, for the AddressSanitizer / UndefinedBehaviorSanitizer
// build of tests/test_sanitizers.py.  Exits non-zero if a result is wrong:
// a malformed input accepted, a valid one refused, a schedule that does not
// cover every nonzero exactly once, or a transpose that is not an involution.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "prep.h"

using namespace pdhcg;

namespace {

struct Csr {
    int64_t rows = 0, cols = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> cj;
    std::vector<double> v;
};

// random CSR with the given row lengths (sorted, distinct columns)
Csr random_csr(std::mt19937_64& rng, int64_t cols, const std::vector<int64_t>& lengths)
{
    Csr M;
    M.rows = (int64_t)lengths.size();
    M.cols = cols;
    M.rp.assign(M.rows + 1, 0);
    std::normal_distribution<double> nd;
    for (int64_t i = 0; i < M.rows; ++i) {
        std::vector<char> used(cols, 0);
        std::vector<int32_t> row;
        std::uniform_int_distribution<int64_t> pick(0, cols - 1);
        while ((int64_t)row.size() < lengths[i]) {
            const int64_t j = pick(rng);
            if (!used[j]) { used[j] = 1; row.push_back((int32_t)j); }
        }
        std::sort(row.begin(), row.end());
        for (int32_t j : row) { M.cj.push_back(j); M.v.push_back(nd(rng)); }
        M.rp[i + 1] = (int64_t)M.cj.size();
    }
    return M;
}

int expect(const char* what, bool ok)
{
    if (!ok) std::printf("FAILED: %s\n", what);
    return ok ? 0 : 1;
}

// every nonzero of [0, nnz) in exactly one schedule item, rows in order
int check_plan(const Csr& M)
{
    std::vector<BlkDesc> blk;
    int nlr = 0, nseg = 0;
    build_plan(M.rows, M.rp.data(), blk, nlr, nseg);
    std::vector<int> seen(M.cj.size(), 0);
    int bad = 0;
    for (const BlkDesc& b : blk) {
        if (b.nrows > ROWS_CAP) ++bad;
        // a single row of up to ROW_PASS_CAP nonzeros may be one item
        if (b.k1 - b.k0 > (b.nrows == 1 ? ROW_PASS_CAP : NNZ_CAP)) ++bad;
        if (b.nrows == 0 && b.nseg > 0 && M.rp[b.row0 + 1] - M.rp[b.row0] <= ROW_PASS_CAP) ++bad;
        if (b.nrows > 0 && (b.k0 != M.rp[b.row0] || b.k1 != M.rp[b.row0 + b.nrows])) ++bad;
        for (int k = b.k0; k < b.k1; ++k) seen[k]++;
    }
    for (int s : seen) bad += s != 1;
    return expect("schedule covers every nonzero once", bad == 0);
}

}  // namespace

int main()
{
    std::mt19937_64 rng(2602);
    int bad = 0;

    // schedules over ragged rows straddling every cap
    std::vector<int64_t> lengths = {0, 1, 2, 255, 256, 257, 2047, 2048, 2049, 5000, 0, 9000, 3, 0};
    for (int i = 0; i < 3000; ++i) lengths.push_back((int64_t)(rng() % 40));
    Csr M = random_csr(rng, 12000, lengths);
    bad += expect("valid CSR accepted", check_csr("M", M.rows, M.cols, M.rp.data(), M.cj.data(), M.v.data()) == 0);
    bad += check_plan(M);
    Csr E;
    E.rows = 0;
    E.cols = 5;
    E.rp = {0};
    bad += check_plan(E);

    // transpose twice is the identity
    std::vector<int64_t> tp, tp2;
    std::vector<int32_t> tj, tj2;
    std::vector<double> tv, tv2;
    transpose(M.rows, M.cols, M.rp.data(), M.cj.data(), M.v.data(), tp, tj, tv);
    transpose(M.cols, M.rows, tp.data(), tj.data(), tv.data(), tp2, tj2, tv2);
    bad += expect("transpose is an involution", tp2 == M.rp && tj2 == M.cj && tv2 == M.v);

    // column parts of a wide matrix: every nonzero once, parts in range
    {
        std::vector<int64_t> L(5000);
        for (auto& x : L) x = 6 + (int64_t)(rng() % 10);
        Csr W = random_csr(rng, 300000, L);
        std::vector<int> prow;
        std::vector<int32_t> pcol;
        std::vector<double> pval;
        std::vector<BlkDesc> blk;
        const bool ok = build_parts(W.rows, W.cols, W.rp.data(), W.cj.data(), W.v.data(), prow, pcol, pval, blk);
        bad += expect("wide matrix partitioned", ok);
        std::vector<int> seen(pcol.size(), 0);
        for (const BlkDesc& b : blk)
            for (int k = b.k0; k < b.k1; ++k) seen[k]++;
        int cover = 0;
        for (int s : seen) cover += s != 1;
        bad += expect("parts cover every nonzero once", cover == 0 && pcol.size() == W.cj.size());
    }

    // malformed inputs are refused
    {
        Csr B = M;
        B.cj[M.rp[5]] = (int32_t)M.cols;   // column out of range (row 5 is not empty)
        bad += expect("column out of range refused",
                      check_csr("B", B.rows, B.cols, B.rp.data(), B.cj.data(), B.v.data()) == QP_ERR_INVALID_ARG);
        B = M;
        std::swap(B.cj[M.rp[4]], B.cj[M.rp[4] + 1]);   // unsorted row
        bad += expect("unsorted row refused",
                      check_csr("B", B.rows, B.cols, B.rp.data(), B.cj.data(), B.v.data()) == QP_ERR_INVALID_ARG);
        B = M;
        B.cj[M.rp[4] + 1] = B.cj[M.rp[4]];   // duplicate
        bad += expect("duplicate column refused",
                      check_csr("B", B.rows, B.cols, B.rp.data(), B.cj.data(), B.v.data()) == QP_ERR_INVALID_ARG);
        B = M;
        B.v[7] = NAN;
        bad += expect("NaN value refused",
                      check_csr("B", B.rows, B.cols, B.rp.data(), B.cj.data(), B.v.data()) == QP_ERR_INVALID_ARG);
        B = M;
        B.rp[3] = B.rp[4] + 1;   // decreasing row pointers
        bad += expect("decreasing row pointers refused",
                      check_csr("B", B.rows, B.cols, B.rp.data(), B.cj.data(), B.v.data()) == QP_ERR_INVALID_ARG);
        bad += expect("NULL row pointer refused",
                      check_csr("B", 3, 3, nullptr, nullptr, nullptr) == QP_ERR_INVALID_ARG);
    }

    // symmetry
    {
        const int64_t n = 800;
        std::vector<int64_t> L(n);
        for (auto& x : L) x = 1 + (int64_t)(rng() % 8);
        Csr H = random_csr(rng, n, L);
        Csr Ht;
        transpose(H.rows, H.cols, H.rp.data(), H.cj.data(), H.v.data(), Ht.rp, Ht.cj, Ht.v);
        // S = H + H' (entries merged row by row)
        Csr S;
        S.rows = S.cols = n;
        S.rp.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t k = H.rp[i]; k < H.rp[i + 1]; ++k) row.push_back({H.cj[k], H.v[k]});
            for (int64_t k = Ht.rp[i]; k < Ht.rp[i + 1]; ++k) row.push_back({Ht.cj[k], Ht.v[k]});
            std::sort(row.begin(), row.end(), [](auto& a, auto& b) { return a.first < b.first; });
            for (size_t q = 0; q < row.size(); ++q) {
                if (q + 1 < row.size() && row[q + 1].first == row[q].first) {
                    row[q + 1].second += row[q].second;
                    continue;
                }
                S.cj.push_back(row[q].first);
                S.v.push_back(row[q].second);
            }
            S.rp[i + 1] = (int64_t)S.cj.size();
        }
        bad += expect("symmetric Q accepted", check_symmetric(n, S.rp.data(), S.cj.data(), S.v.data()) == 0);
        bad += expect("non-symmetric Q refused",
                      check_symmetric(n, H.rp.data(), H.cj.data(), H.v.data()) == QP_ERR_NOT_SYMMETRIC);
    }

    // vectors and boxes
    {
        std::vector<double> a = {1.0, INFINITY, -2.0}, l = {0.0, -INFINITY, 1.0}, u = {1.0, 2.0, 1.0};
        bad += expect("infinite entry refused", check_vec("a", 3, a.data(), false) == QP_ERR_INVALID_ARG);
        bad += expect("infinite entry allowed", check_vec("a", 3, a.data(), true) == 0);
        bad += expect("valid box accepted", check_bounds("box", 3, l.data(), u.data()) == 0);
        u[2] = 0.5;
        bad += expect("crossed box refused", check_bounds("box", 3, l.data(), u.data()) == QP_ERR_INVALID_ARG);
        bad += expect("NULL vector refused", check_vec("a", 3, nullptr, false) == QP_ERR_INVALID_ARG);
    }

    // box storage classes: one pair, byte classes, arrays
    {
        std::vector<unsigned char> cls;
        std::vector<double> tl, tu;
        std::vector<double> lv(1000, 0.0), uv(1000, 10.0);
        bad += expect("one pair", classify_bounds(lv, uv, cls, tl, tu) == 1 && tl.size() == 1);
        for (int i = 0; i < 1000; ++i) uv[i] = 1.0 + (i % 200);
        const int mode = classify_bounds(lv, uv, cls, tl, tu);
        int same = 0;
        for (int i = 0; i < 1000; ++i) same += tl[cls[i]] == lv[i] && tu[cls[i]] == uv[i];
        bad += expect("byte classes", mode == 2 && same == 1000);
        for (int i = 0; i < 1000; ++i) uv[i] = 1.0 + i;
        bad += expect("arrays", classify_bounds(lv, uv, cls, tl, tu) == 0);
    }

    std::printf("prep driver: %d failure(s)\n", bad);
    return bad ? 1 : 0;
}
