// Dispatch of the last-axis kernels, float instantiations.
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

// The direct passes (lanes index-fastest) of 128- and 256-entry rows, with the
// rows per block of variant 3 (the half tiles).
template <int MODE, int HH>
static hipError_t go_direct1(const RowArgs<float, float>& a, int64_t nb, hipStream_t s) {
  constexpr int R = tile_rows<float>(HH, 3);
  hipLaunchKernelGGL((row_direct_kernel<MODE, HH, R>), dim3((unsigned)nb), dim3(R * (HH / 16)), 0, s, a);
  return hipGetLastError();
}
template <int MODE>
static hipError_t go_direct(int H, const RowArgs<float, float>& a, int64_t nb, hipStream_t s) {
  return H == 128 ? go_direct1<MODE, 128>(a, nb, s) : go_direct1<MODE, 256>(a, nb, s);
}

hipError_t launch_row_f32(int mode, int H, int v, const void* args, int64_t nb, hipStream_t s) {
  const RowArgs<float, float>& a = *static_cast<const RowArgs<float, float>*>(args);
  const bool direct = v == 3 && (H == 128 || H == 256);
  switch (mode) {
    case ROW_INIT: return direct ? go_direct<ROW_INIT>(H, a, nb, s) : go<float, float, ROW_INIT, 0>(H, a, nb, s);
    case ROW_LOOP:
      if (v == 3) return direct ? go_direct<ROW_LOOP>(H, a, nb, s) : go<float, float, ROW_LOOP, 1>(H, a, nb, s);
      return v == 2 ? go<float, float, ROW_LOOP, 2>(H, a, nb, s)
                    : (v ? go<float, float, ROW_LOOP, 1>(H, a, nb, s) : go<float, float, ROW_LOOP, 0>(H, a, nb, s));
    case ROW_FINAL: return direct ? go_direct<ROW_FINAL>(H, a, nb, s) : go<float, float, ROW_FINAL, 0>(H, a, nb, s);
    case ROW_BINIT: return direct ? go_direct<ROW_BINIT>(H, a, nb, s) : go<float, float, ROW_BINIT, 0>(H, a, nb, s);
    case ROW_BLOOP: return direct ? go_direct<ROW_BLOOP>(H, a, nb, s) : go<float, float, ROW_BLOOP, 0>(H, a, nb, s);
    case ROW_BFINAL:
      return direct ? go_direct<ROW_BFINAL>(H, a, nb, s) : go<float, float, ROW_BFINAL, 0>(H, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
