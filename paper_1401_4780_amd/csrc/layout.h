// Row record layout of the asynchronous randomized Kaczmarz library: plain
// C++ (no HIP), shared by the host packing code and the kernels.
#pragma once

#include <stdint.h>

#include "../../include/asyrk.h"

namespace asyrk {

// ---------------------------------------------------------------------------
// Row record layout in device memory.
//
// One record per row: a header, then the row's (column, value) pairs grouped
// in "units" so that one lane reads a unit with 16-byte loads:
//   F32 : unit = int32 col[4], float  val[4]      (32 B, 4 entries)
//   BF16: unit = int32 col[8], bf16   val[8]      (48 B, 8 entries)
//   F64 : unit = int32 col[4], double val[4]      (48 B, 4 entries)
// The last unit of a row is padded with (0, 0) entries that no kernel uses.
// Header (F32/BF16 sweeps):  { float b_i; float 1/w_i; u32 T; i32 alias }    16 B
// Header (F64 sweeps):       { double b_i; double 1/w_i; u32 T; i32 alias; pad } 32 B
// with w_i = ||a_i||^2.  Row k is chosen from alias bucket k when u2 < T,
// otherwise row `alias`; buckets that always keep their row alias themselves.
// ---------------------------------------------------------------------------
struct HdrF32 {
    float b;
    float inv_w;
    uint32_t thresh;
    int32_t alias;
};
struct HdrF64 {
    double b;
    double inv_w;
    uint32_t thresh;
    int32_t alias;
    uint64_t pad;
};
static_assert(sizeof(HdrF32) == 16, "header");
static_assert(sizeof(HdrF64) == 32, "header");

template <int VK> struct VT;
template <> struct VT<ASYRK_F32> {
    using val_t = float;
    using x_t = float;
    using hdr_t = HdrF32;
    static constexpr int U = 4;         // entries per unit
    static constexpr int UB = 32;       // bytes per unit
    static constexpr int COLB = 16;     // bytes of column indices per unit
    static constexpr int HB = 16;       // header bytes
    static constexpr int VB = 4;        // bytes per stored value
};
template <> struct VT<ASYRK_BF16> {
    using val_t = uint16_t;
    using x_t = float;
    using hdr_t = HdrF32;
    static constexpr int U = 8;
    static constexpr int UB = 48;
    static constexpr int COLB = 32;
    static constexpr int HB = 16;
    static constexpr int VB = 2;
};
template <> struct VT<ASYRK_F64> {
    using val_t = double;
    using x_t = double;
    using hdr_t = HdrF64;
    static constexpr int U = 4;
    static constexpr int UB = 48;
    static constexpr int COLB = 16;
    static constexpr int HB = 32;
    static constexpr int VB = 8;
};

// Per-row locator for systems whose rows differ in length: record offset in
// 16-byte units and the row length.
struct RowLoc {
    uint32_t off16;
    uint32_t nnz;
};

// Record geometry of one value dtype, for host code.
struct Geom {
    int U, UB, COLB, HB, VB;
};
inline Geom geom_of(int vk) {
    switch (vk) {
        case ASYRK_F32: return Geom{4, 32, 16, 16, 4};
        case ASYRK_BF16: return Geom{8, 48, 32, 16, 2};
        default: return Geom{4, 48, 16, 32, 8};
    }
}

}  // namespace asyrk
