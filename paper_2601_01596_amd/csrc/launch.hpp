// Host-side dispatch from runtime lengths to the templated kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace ffcz {

// Columns per block used by the strided-axis kernels of this dtype and length.
int col_block_cols(int dtype, int L);
// Rows per block of the last-axis kernels computing in this dtype.
int row_block_rows(int dtype, int H);

// dtype 0: float, 1: double.  args points to a ColArgs<T>.
hipError_t launch_col(int dtype, int mode, int L, const void* args, int64_t nblocks, hipStream_t s);
// tdtype: compute type (0 float, 1 double); iodtype: storage type of the real fields.
hipError_t launch_row(int tdtype, int iodtype, int mode, int H, const void* args, int64_t nblocks,
                      hipStream_t s);

}  // namespace ffcz
