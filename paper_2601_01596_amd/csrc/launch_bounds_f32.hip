// Dispatch of the passes against pointwise bounds, float fields (default tiles; the FP64
// verification's last-axis pass on the verification plan's tiles).
#include "kernels_col.hpp"
#include "kernels_row.hpp"
#include "launch.hpp"

namespace ffcz {

template <typename T, typename TIO, int MODE, int V>
static hipError_t go_row(int H, const RowArgs<T, TIO>& a, int64_t nb, hipStream_t s) {
  switch (H) {
#define FFCZ_CASE(HH)                                                                          \
  case HH: {                                                                                   \
    constexpr int R = tile_rows<T>(HH, V);                                                     \
    constexpr int EE = row_E(HH, V);                                                           \
    hipLaunchKernelGGL((row_kernel<T, TIO, HH, R, MODE, EE>), dim3((unsigned)nb), dim3(R * (HH / EE)), 0, s, a); \
    return hipGetLastError();                                                                  \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int MODE>
static hipError_t go_col(int L, const ColArgs<T>& a, int64_t nb, hipStream_t s) {
  switch (L) {
#define FFCZ_CASE(LL)                                                                          \
  case LL: {                                                                                   \
    constexpr int C = tile_cols<T>(LL, 0);                                                     \
    hipLaunchKernelGGL((col_kernel<T, LL, C, MODE>), dim3((unsigned)nb), dim3(C * (LL / pick_E(LL))), 0, s, a); \
    return hipGetLastError();                                                                  \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

// Last-axis passes of a float field: the loop's modes compute in float; ROW_VERIFYP computes in
// double on the tiles of plan variant vv (the verification plan).
hipError_t launch_bounds_row_f32(int mode, int H, int vv, const void* args, int64_t nb, hipStream_t s) {
  if (mode == ROW_VERIFYP) {
    const RowArgs<double, float>& a = *static_cast<const RowArgs<double, float>*>(args);
    return vv == 2 ? go_row<double, float, ROW_VERIFYP, 2>(H, a, nb, s) : go_row<double, float, ROW_VERIFYP, 0>(H, a, nb, s);
  }
  const RowArgs<float, float>& a = *static_cast<const RowArgs<float, float>*>(args);
  switch (mode) {
    case ROW_INITP: return go_row<float, float, ROW_INITP, 0>(H, a, nb, s);
    case ROW_LOOPP: return go_row<float, float, ROW_LOOPP, 0>(H, a, nb, s);
    case ROW_FINALP: return go_row<float, float, ROW_FINALP, 0>(H, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bounds_col_f32(int mode, int L, const void* args, int64_t nb, hipStream_t s) {
  if (mode != COL_XPASSP) return hipErrorInvalidValue;
  return go_col<float, COL_XPASSP>(L, *static_cast<const ColArgs<float>*>(args), nb, s);
}

}  // namespace ffcz
