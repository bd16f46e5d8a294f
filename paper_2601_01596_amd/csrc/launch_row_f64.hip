// Dispatch of the last-axis kernels, double instantiations.
#include "kernels_row.hpp"
#include "launch.hpp"

namespace ffcz {

template <typename T, typename TIO, int MODE>
static hipError_t go(int H, const RowArgs<T, TIO>& a, int64_t nb, hipStream_t s) {
  switch (H) {
#define FFCZ_CASE(HH)                                                                  \
  case HH: {                                                                           \
    constexpr int R = pick_rows<T>(HH);                                                   \
    constexpr int NT = R * (HH / pick_E_row(HH));                                          \
    hipLaunchKernelGGL((row_kernel<T, TIO, HH, R, MODE>), dim3((unsigned)nb), dim3(NT), 0, s, a); \
    return hipGetLastError();                                                          \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row_f64(int mode, int H, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<double, double>& a = *static_cast<const RowArgs<double, double>*>(args);
  switch (mode) {
    case ROW_INIT: return go<double, double, ROW_INIT>(H, a, nb, s);
    case ROW_LOOP: return go<double, double, ROW_LOOP>(H, a, nb, s);
    case ROW_FINAL: return go<double, double, ROW_FINAL>(H, a, nb, s);
    case ROW_VERIFY: return go<double, double, ROW_VERIFY>(H, a, nb, s);
    case ROW_BINIT: return go<double, double, ROW_BINIT>(H, a, nb, s);
    case ROW_BLOOP: return go<double, double, ROW_BLOOP>(H, a, nb, s);
    case ROW_BFINAL: return go<double, double, ROW_BFINAL>(H, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

// FP64 verification of an FP32 output: compute in double, read float fields.
hipError_t launch_row_verify_f32io(int H, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<double, float>& a = *static_cast<const RowArgs<double, float>*>(args);
  return go<double, float, ROW_VERIFY>(H, a, nb, s);
}

}  // namespace ffcz
