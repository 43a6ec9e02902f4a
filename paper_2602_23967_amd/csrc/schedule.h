// schedule.h -- the SpMV work schedule's constants and item layout, shared
// by the host-side schedule builder (prep.cpp), the kernels and the host
// driver.  No HIP types: prep.cpp also builds with a plain C++ compiler.
#pragma once

#include <stdint.h>

namespace pdhcg {

constexpr int TPB = 256;        // threads per block for every kernel
#ifndef PDHCG_NNZ_CAP
#define PDHCG_NNZ_CAP 2048
#endif
#ifndef PDHCG_PART_ROWS_CAP
#define PDHCG_PART_ROWS_CAP 1024
#endif
constexpr int NNZ_CAP = PDHCG_NNZ_CAP;   // nonzeros staged in LDS per row block
constexpr int ROWS_CAP = 256;   // rows per row block (one thread per row at most)
// a row of more than NNZ_CAP and at most ROW_PASS_CAP nonzeros is summed by
// one block in strided passes (no segments, so no finishing step completes
// it); longer rows are split into NNZ_CAP-sized segments
constexpr int ROW_PASS_CAP = 4 * NNZ_CAP;
// blocks of an elementwise pass at most: 4 per CU; each thread then takes
// several elements (1024 measured 1.3 % faster on the n = 1e6 QP than 2048,
// and 0.3 % faster than 512; the other workloads do not change)
constexpr int VEC_GRID_MAX = 1024;
// XCD-aware column partitioning: an operand larger than PART_MIN_COLS
// doubles is split into NPARTS contiguous column parts; block b of the
// product works on part b % NPARTS, which on gfx950's round-robin dispatch of
// blocks to its 8 XCDs keeps each XCD's gathers inside one part (1/4 of the
// operand, L2-resident).  4 parts measured faster than 2 or 8 on the
// 1e6 x 1e6 product with 11 nonzeros per row (71 us against 77 and 101:
// 2 parts' 4 MB segments thrash the 4 MB L2, 8 parts double the partial row
// traffic); the gathers themselves reach about 250 G/s with 2 to 16 parts
// and 120 G/s with none.
#ifndef PDHCG_NPARTS
#define PDHCG_NPARTS 4
#endif
constexpr int NPARTS = PDHCG_NPARTS;
constexpr int PART_MIN_COLS = 262144;
// and with at least this many nonzeros per row on average: a part of a
// sparser matrix holds about one nonzero per row, and the partial row sums
// (NPARTS x 8 bytes per row, written and read back) cost more than the
// gathers save (A' of the large sparse QP, 4 per row: 49 us whole against
// 62 us in parts; A, 8 per row: 55 us in parts against 59 us whole)
#ifndef PDHCG_PART_MIN_NNZ_ROW
#define PDHCG_PART_MIN_NNZ_ROW 6
#endif
constexpr int PART_MIN_NNZ_ROW = PDHCG_PART_MIN_NNZ_ROW;
constexpr int PART_ROWS_CAP = PDHCG_PART_ROWS_CAP;   // rows per block of a column part
#ifndef PDHCG_FIN_T
#define PDHCG_FIN_T 256
#endif
// threads of the one-block finishing kernels (256 against 512, with 1024
// partials per product: the n = 1e6 QP 0.2 %, the portfolio 0.8 % and the
// n = 1000 QP 2.4 % faster per solve; 512 had won when the elementwise
// passes left 2048 partials)
constexpr int FIN_T = PDHCG_FIN_T;
// long rows the finishing kernel completes with the whole block: all of them
// when there are at most LR_COOP, else those with more than LR_SEG_SERIAL
// segments (the others one thread per row)
constexpr int LR_COOP = 32;
constexpr int LR_SEG_SERIAL = 8;

// One work item of the row-block SpMV schedule.
//   nrows > 0            rows [row0, row0+nrows), nonzeros [k0, k1); for a
//                        column-partitioned matrix `lr` is the column part;
//                        k1 - k0 > NNZ_CAP only for a single row (nrows == 1)
//                        of at most ROW_PASS_CAP nonzeros
//   nrows == 0, nseg > 0 segment `seg` of long row row0 (nonzeros [k0, k1));
//                        its partial sum lands in seg_part[seg_base + seg] and
//                        the finishing kernel completes the row (long row lr)
//   nrows == 0, nseg == 0 empty item (keeps a grid of >= 1 block)
struct BlkDesc {
    int row0, nrows, k0, k1;
    int lr, seg, nseg, seg_base;
};

}  // namespace pdhcg
