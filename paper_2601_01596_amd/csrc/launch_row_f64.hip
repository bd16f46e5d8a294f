// Dispatch of the last-axis kernels, double instantiations.
#include "kernels_row.hpp"
#include "launch.hpp"

namespace ffcz {

// V: tile variant (rows per block = pick_rows >> V), chosen per size by the tuner
template <typename T, typename TIO, int MODE, int V>
static hipError_t go(int H, const RowArgs<T, TIO>& a, int64_t nb, hipStream_t s) {
  switch (H) {
#define FFCZ_CASE(HH)                                                                  \
  case HH: {                                                                           \
    constexpr int R = tile_rows<T>(HH, V);                                                \
    constexpr int EE = row_E(HH, V);                                                       \
    constexpr int NT = R * (HH / EE);                                                      \
    hipLaunchKernelGGL((row_kernel<T, TIO, HH, R, MODE, EE>), dim3((unsigned)nb), dim3(NT), 0, s, a); \
    return hipGetLastError();                                                          \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row_f64(int mode, int H, int v, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<double, double>& a = *static_cast<const RowArgs<double, double>*>(args);
  switch (mode) {
    case ROW_INIT: return go<double, double, ROW_INIT, 0>(H, a, nb, s);
    case ROW_LOOP:
      // variant 3 (FP32 only) falls back to variant 1, whose tiles it shares
      return v == 2 ? go<double, double, ROW_LOOP, 2>(H, a, nb, s)
                    : (v ? go<double, double, ROW_LOOP, 1>(H, a, nb, s) : go<double, double, ROW_LOOP, 0>(H, a, nb, s));
    case ROW_FINAL: return v == 2 ? go<double, double, ROW_FINAL, 2>(H, a, nb, s) : go<double, double, ROW_FINAL, 0>(H, a, nb, s);
    case ROW_FINALV: return go<double, double, ROW_FINALV, 2>(H, a, nb, s);
    case ROW_VERIFY: return v == 2 ? go<double, double, ROW_VERIFY, 2>(H, a, nb, s) : go<double, double, ROW_VERIFY, 0>(H, a, nb, s);
    case ROW_BINIT: return go<double, double, ROW_BINIT, 0>(H, a, nb, s);
    case ROW_BLOOP: return go<double, double, ROW_BLOOP, 0>(H, a, nb, s);
    case ROW_BFINAL: return go<double, double, ROW_BFINAL, 0>(H, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

// FP64 verification of an FP32 output: compute in double, read float fields.
hipError_t launch_row_f64_f32io(int mode, int H, int v, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<double, float>& a = *static_cast<const RowArgs<double, float>*>(args);
  if (mode != ROW_VERIFY) return hipErrorInvalidValue;
  return v == 2 ? go<double, float, ROW_VERIFY, 2>(H, a, nb, s) : go<double, float, ROW_VERIFY, 0>(H, a, nb, s);
}

}  // namespace ffcz
