// qt_tune.h -- tile-shape decisions of the autotuner (host side).
//
// Decisions are kept in a process-wide table keyed by kernel family, precision and size bucket
// (for CSR, the bucket of the whole CSR group of a plan, which shares one launch shape).  The
// table can be saved to and loaded from a small JSON file.
#pragma once
#include <cstdint>
#include <string>

namespace qt {

struct CsrShape {
    int lpr = 8;  // lanes per row group
    int rg = 1;   // rows per lane group
    int xcd = 0;   // 1: XCD-contiguous block order
    int keep = 0;  // 1: temporal matrix loads, the matrix may stay in L2 / MALL across launches;
                   // 2: as 1 with 16-byte loads of runs of 4 stored entries
};

// size bucket of a CSR right-hand side: log2 of the rows, rounded mean row length
std::string csr_tune_key(int32_t prec, int64_t rows, double mean_row);
std::string dense_tune_key(int32_t prec, int np);

bool tune_lookup_csr(const std::string &key, CsrShape *out);
void tune_store_csr(const std::string &key, CsrShape s);
bool tune_lookup_dense(const std::string &key, int *waves);
void tune_store_dense(const std::string &key, int waves);

// heuristic shapes used when the table has no entry
CsrShape csr_default_shape(int64_t rows, double mean_row);
int dense_default_waves(int np, int32_t prec);

// Candidate CSR shapes the autotuner measures (both matrix load kinds).  single: include the
// XCD-contiguous block order, which only single-problem plans use: with several problems of
// unequal step counts, an XCD whose problems have finished would sit idle while the others still
// work through theirs.
int csr_candidates(CsrShape *out, int max, bool single);

}  // namespace qt
