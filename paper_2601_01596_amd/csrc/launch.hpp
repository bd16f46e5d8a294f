// Host-side dispatch from runtime lengths to the templated kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace ffcz {

// Columns per block used by the strided-axis kernels of this dtype, length and
// tile variant (only the loop modes COL_FWD / COL_INV / COL_XPASS have variant 1).
int col_block_cols(int dtype, int L, int v);
// Rows per block of the last-axis kernels computing in this dtype (plan variants
// 1 and 2 exist for ROW_LOOP, variant 2 for ROW_VERIFY and, on FP64 fields, for
// ROW_FINAL and ROW_FINALV).
int row_block_rows(int dtype, int H, int v);

// dtype 0: float, 1: double.  args points to a ColArgs<T>.
hipError_t launch_col(int dtype, int mode, int L, int v, const void* args, int64_t nblocks, hipStream_t s);

}  // namespace ffcz
