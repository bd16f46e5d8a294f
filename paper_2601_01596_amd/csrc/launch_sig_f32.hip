// Dispatch of the per-signal kernels (float data).
#include "kernels_sig.hpp"
#include "launch.hpp"

namespace ffcz {

template <typename T, typename TIO, int MODE>
static hipError_t go(int lgMc, const SigArgs<T>& a, int nb, hipStream_t s) {
  switch (lgMc) {
#define FFCZ_CASE(LG, MA, MB)                                                                       \
  case LG: {                                                                                         \
    hipLaunchKernelGGL((sig_kernel<T, TIO, MA, MB, MODE>), dim3((unsigned)nb), dim3((SigGeom<T, MA, MB>::NT)), 0, s, a); \
    return hipGetLastError();                                                                       \
  }
    FFCZ_CASE(2, 2, 2) FFCZ_CASE(3, 4, 2) FFCZ_CASE(4, 4, 4) FFCZ_CASE(5, 8, 4) FFCZ_CASE(6, 8, 8)
    FFCZ_CASE(7, 16, 8) FFCZ_CASE(8, 16, 16) FFCZ_CASE(9, 32, 16) FFCZ_CASE(10, 32, 32)
    FFCZ_CASE(11, 64, 32) FFCZ_CASE(12, 64, 64) FFCZ_CASE(13, 128, 64) FFCZ_CASE(14, 128, 128)
    FFCZ_CASE(15, 256, 128) FFCZ_CASE(16, 256, 256) FFCZ_CASE(17, 512, 256) FFCZ_CASE(18, 512, 512)
    FFCZ_CASE(19, 1024, 512) FFCZ_CASE(20, 1024, 1024)
#undef FFCZ_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sig_f32(int mode, int lgMc, const void* args, int nb, hipStream_t s) {
  // the FP32 loop; its FP64 verification (double compute, float data)
  if (mode == SIG_RUN) return go<float, float, SIG_RUN>(lgMc, *static_cast<const SigArgs<float>*>(args), nb, s);
  if (mode == SIG_VERIFY) return go<double, float, SIG_VERIFY>(lgMc, *static_cast<const SigArgs<double>*>(args), nb, s);
  return hipErrorInvalidValue;
}

}  // namespace ffcz
