// Dispatch of the last-axis kernels, float instantiations.
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

hipError_t launch_row_f32(int mode, int H, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<float, float>& a = *static_cast<const RowArgs<float, float>*>(args);
  switch (mode) {
    case ROW_INIT: return go<float, float, ROW_INIT>(H, a, nb, s);
    case ROW_LOOP: return go<float, float, ROW_LOOP>(H, a, nb, s);
    case ROW_FINAL: return go<float, float, ROW_FINAL>(H, a, nb, s);
    case ROW_BINIT: return go<float, float, ROW_BINIT>(H, a, nb, s);
    case ROW_BLOOP: return go<float, float, ROW_BLOOP>(H, a, nb, s);
    case ROW_BFINAL: return go<float, float, ROW_BFINAL>(H, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
