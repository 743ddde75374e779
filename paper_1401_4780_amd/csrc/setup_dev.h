// Device-side setup of a system whose CSR arrays already sit in device memory
// (setup_dev.hip): validation, row weights and column statistics in one pass
// over the entries, then the packed row records written straight from the
// caller's arrays.  The record plan and the alias table stay on the host
// (setup.cpp), which sees only row_ptr and the row weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"
#include "setup.h"  // RowAux

namespace asyrk {

// Bits of the validation flag word.
enum : uint32_t {
    kBadEntry = 1u,   // a column out of range or not increasing within its row, or a non-finite value
    kBadRhs = 2u,     // a non-finite b_i
};

// Rows 0..m-1 of a CSR whose row_ptr the host has checked (row_ptr[0] = 0,
// non-decreasing, row_ptr[m] = nnz): w_i = sum of v^2 over the row in CSR
// order (FP64 from the stored values, no fused multiply-add, the host's exact
// sum), per-column entry counts and sums of squares (atomics: the sums equal
// the host's up to rounding order), and kBadEntry / kBadRhs or-ed into *flags.
// col_cnt, col_sq and *flags must be zero on entry.
hipError_t launch_scan_rows_dev(int vk, int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                                const void *vals, const double *b, double *w, uint32_t *col_cnt, double *col_sq,
                                uint32_t *flags, hipStream_t st);
// kBadRhs or-ed into *flags if any of v[0..n-1] is not finite.
hipError_t launch_check_finite_dev(const double *v, int64_t n, uint32_t *flags, hipStream_t st);
// out[0] = max_j col_cnt[j], out[1] = bits of max_j col_sq[j]; out zero on entry.
hipError_t launch_col_max_dev(const uint32_t *col_cnt, const double *col_sq, int64_t n, unsigned long long *out,
                              hipStream_t st);
// Records of rows 0..m-1, byte for byte what the host packing writes: header
// from b and aux, whole units, the last one padded with (0, 0) entries, and
// (loc == nullptr: rows of equal length at `stride` bytes) zeros up to the
// stride; with loc, row i starts at byte 16 * loc[i].off16.
hipError_t launch_write_records_dev(int vk, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                    const void *vals, const double *b, const RowAux *aux, int64_t stride,
                                    const RowLoc *loc, uint8_t *rec, hipStream_t st);

}  // namespace asyrk
