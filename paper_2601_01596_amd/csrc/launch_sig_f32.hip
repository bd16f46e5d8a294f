// Dispatch of the per-signal kernels on float data: the FP32 loop (one-block and
// tiled passes) and the one-block FP64 verification.
#include "launch.hpp"
#include "sig_dispatch.hpp"

namespace ffcz {

hipError_t launch_sig_f32(int mode, int lgMc, const void* args, int nsig, hipStream_t s) {
  const SigArgs<float>& a = *static_cast<const SigArgs<float>*>(args);
  switch (mode) {
    case SIG_RUN: return sig_go<float, float, SIG_RUN>(lgMc, a, nsig, s);
    case SIG_RUNL: return sig_go<float, float, SIG_RUNL>(lgMc, a, nsig, s);
    case SIG_VERIFY:
      return sig_go<double, float, SIG_VERIFY>(lgMc, *static_cast<const SigArgs<double>*>(args), nsig, s);
    case SIGT_EPS0: return sig_go<float, float, SIGT_EPS0>(lgMc, a, nsig, s);
    case SIGT_CIN: return sig_go<float, float, SIGT_CIN>(lgMc, a, nsig, s);
    case SIGT_RMUL: return sig_go<float, float, SIGT_RMUL>(lgMc, a, nsig, s);
    case SIGT_RMULI: return sig_go<float, float, SIGT_RMULI>(lgMc, a, nsig, s);
    case SIGT_RCHECK: return sig_go<float, float, SIGT_RCHECK>(lgMc, a, nsig, s);
    case SIGT_CCHECK: return sig_go<float, float, SIGT_CCHECK>(lgMc, a, nsig, s);
    case SIGT_CSPAT: return sig_go<float, float, SIGT_CSPAT>(lgMc, a, nsig, s);
    case SIGT_Y: return sig_go<float, float, SIGT_Y>(lgMc, a, nsig, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
