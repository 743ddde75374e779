// Host-side system setup (setup.cpp): validation, row weights, alias table
// and record packing.  Plain C++, no HIP.
#pragma once

#include <stdint.h>

#include <vector>

#include "layout.h"

namespace asyrk {

struct SetupResult {
    std::vector<double> w;     // ||a_i||^2, FP64 from the stored values
    int64_t nnz = 0;
    int64_t mu = 0;            // max row length
    int64_t nu = 0;            // max column count
    int64_t fixed_nnz = 0;     // common row length or 0
    double fro2 = 0.0;         // sum of w
    double max_col_norm2 = 0.0;  // max_j ||column j||^2
    int64_t stride = 0;        // record stride (fixed rows)
    std::vector<RowLoc> loc;   // per-row locators (rows of different length)
    std::vector<uint8_t> rec;  // packed records
};

// Augmented consistent system for least squares (inconsistent A x = b):
// [[0, phi A^T], [A, -zeta I]] z = [phi A^T b; 0], z = (x, y) of length n + m.
struct AugCSR {
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<uint8_t> vals;  // in the storage dtype of A
    std::vector<double> b;
};
asyrk_status build_augmented(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const void *vals, int vk, const double *b, double zeta, double phi, AugCSR &out);

asyrk_status validate_system(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const void *vals, int vk, const double *b, SetupResult &out);
// Alias table of the weights w[0..m-1] into thresh and alias (m entries each,
// caller memory; see setup.cpp for the construction).  total must be the sum
// of w taken left to right (validate_system's fro2).
void build_alias(const double *w, int64_t m, double total, uint32_t *thresh, int32_t *alias);
void build_alias(const std::vector<double> &w, std::vector<uint32_t> &thresh,
                 std::vector<int32_t> &alias);

// Per-row values the host derives from the row weights for records written
// on the device: 1/w_i and the alias bucket of row i.
struct RowAux {
    double inv_w;
    uint32_t thresh;
    int32_t alias;
};
static_assert(sizeof(RowAux) == 16, "RowAux");
// aux[i] = {1 / w[i], thresh[i], alias[i]} for i < m.
void row_aux(const double *w, int64_t m, const uint32_t *thresh, const int32_t *alias, RowAux *aux);
// Alias table, layout and records in res.rec.
asyrk_status pack_records(int64_t m, const int64_t *row_ptr, const int32_t *col, const void *vals,
                          int vk, const double *b, SetupResult &res);
// The two halves of pack_records for callers that place the records
// themselves: plan_records fixes the layout of a validated system (res.stride,
// or res.loc for rows of different length) and its size in bytes;
// write_records fills dst (that many bytes) completely, padding included.
asyrk_status plan_records(int64_t m, const int64_t *row_ptr, int vk, SetupResult &res, int64_t *total_bytes);
void write_records(int64_t m, const int64_t *row_ptr, const int32_t *col, const void *vals, int vk,
                   const double *b, const SetupResult &res, const uint32_t *thresh, const int32_t *alias,
                   uint8_t *dst);

}  // namespace asyrk
