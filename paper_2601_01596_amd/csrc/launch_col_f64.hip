// Dispatch of the strided-axis kernels, double instantiations.
#include "kernels_col.hpp"
#include "launch.hpp"

namespace ffcz {

// V: tile variant (columns per block = pick_C >> V), chosen per size by the tuner
template <int MODE, int V>
static hipError_t go(int L, const ColArgs<double>& a, int64_t nb, hipStream_t s) {
  switch (L) {
#define FFCZ_CASE(LL)                                                               \
  case LL: {                                                                        \
    constexpr int C = tile_cols<double>(LL, V);                                          \
    constexpr int NT = C * (LL / pick_E(LL));                                       \
    hipLaunchKernelGGL((col_kernel<double, LL, C, MODE>), dim3((unsigned)nb), dim3(NT), 0, s, a); \
    return hipGetLastError();                                                       \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col_f64(int mode, int L, int v, const void* args, int64_t nb, hipStream_t s) {
  const ColArgs<double>& a = *static_cast<const ColArgs<double>*>(args);
  switch (mode) {
    case COL_FWD: return v ? go<COL_FWD, 1>(L, a, nb, s) : go<COL_FWD, 0>(L, a, nb, s);
    case COL_INV: return v ? go<COL_INV, 1>(L, a, nb, s) : go<COL_INV, 0>(L, a, nb, s);
    case COL_XPASS: return v ? go<COL_XPASS, 1>(L, a, nb, s) : go<COL_XPASS, 0>(L, a, nb, s);
    case COL_XBACK: return go<COL_XBACK, 0>(L, a, nb, s);
    case COL_FWD_NS: return go<COL_FWD_NS, 0>(L, a, nb, s);
    case COL_INV_NS: return go<COL_INV_NS, 0>(L, a, nb, s);
    case COL_VERIFY: return go<COL_VERIFY, 0>(L, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
