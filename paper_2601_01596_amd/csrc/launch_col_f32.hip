// Dispatch of the strided-axis kernels, float instantiations.
#include "kernels_col.hpp"
#include "launch.hpp"

namespace ffcz {

template <int MODE>
static hipError_t go(int L, const ColArgs<float>& a, int64_t nb, hipStream_t s) {
  switch (L) {
#define FFCZ_CASE(LL)                                                               \
  case LL: {                                                                        \
    constexpr int C = pick_C<float>(LL);                                              \
    constexpr int NT = C * (LL / pick_E(LL));                                       \
    hipLaunchKernelGGL((col_kernel<float, LL, C, MODE>), dim3((unsigned)nb), dim3(NT), 0, s, a); \
    return hipGetLastError();                                                       \
  }
    FFCZ_CASE(1) FFCZ_CASE(2) FFCZ_CASE(4) FFCZ_CASE(8) FFCZ_CASE(16) FFCZ_CASE(32)
    FFCZ_CASE(64) FFCZ_CASE(128) FFCZ_CASE(256) FFCZ_CASE(512) FFCZ_CASE(1024) FFCZ_CASE(2048)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col_f32(int mode, int L, const void* args, int64_t nb, hipStream_t s) {
  const ColArgs<float>& a = *static_cast<const ColArgs<float>*>(args);
  switch (mode) {
    case COL_FWD: return go<COL_FWD>(L, a, nb, s);
    case COL_INV: return go<COL_INV>(L, a, nb, s);
    case COL_XPASS: return go<COL_XPASS>(L, a, nb, s);
    case COL_XBACK: return go<COL_XBACK>(L, a, nb, s);
    case COL_FWD_NS: return go<COL_FWD_NS>(L, a, nb, s);
    case COL_INV_NS: return go<COL_INV_NS>(L, a, nb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
