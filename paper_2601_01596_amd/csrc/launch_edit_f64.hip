// Dispatch of the passes with edit bookkeeping and of the decoder's closing pass,
// double instantiations (default tiles only).
#include "kernels_col.hpp"
#include "kernels_row.hpp"
#include "launch.hpp"

namespace ffcz {

template <int MODE>
static hipError_t go_row(int H, const RowArgs<double, double>& a, int64_t nb, hipStream_t s) {
  switch (H) {
#define FFCZ_CASE(HH)                                                                          \
  case HH: {                                                                                   \
    constexpr int R = tile_rows<double>(HH, 0);                                                   \
    constexpr int EE = row_E(HH, 0);                                                           \
    hipLaunchKernelGGL((row_kernel<double, double, HH, R, MODE, EE>), dim3((unsigned)nb), dim3(R * (HH / EE)), 0, s, a); \
    return hipGetLastError();                                                                  \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
static hipError_t go_col(int L, const ColArgs<double>& a, int64_t nb, hipStream_t s) {
  switch (L) {
#define FFCZ_CASE(LL)                                                                          \
  case LL: {                                                                                   \
    constexpr int C = tile_cols<double>(LL, 0);                                                   \
    hipLaunchKernelGGL((col_kernel<double, LL, C, MODE>), dim3((unsigned)nb), dim3(C * (LL / pick_E(LL))), 0, s, a); \
    return hipGetLastError();                                                                  \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edit_row_f64(int mode, int H, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<double, double>& a = *static_cast<const RowArgs<double, double>*>(args);
  switch (mode) {
    case ROW_INITE: return go_row<ROW_INITE>(H, a, nb, s);
    case ROW_LOOPE: return go_row<ROW_LOOPE>(H, a, nb, s);
    case ROW_DECODE: return go_row<ROW_DECODE>(H, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edit_col_f64(int mode, int L, const void* args, int64_t nb, hipStream_t s) {
  const ColArgs<double>& a = *static_cast<const ColArgs<double>*>(args);
  switch (mode) {
    case COL_XEDIT: return go_col<COL_XEDIT>(L, a, nb, s);
    case COL_XUNDO: return go_col<COL_XUNDO>(L, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
