// Dispatch of the per-signal kernels computing in double: the FP64 one-block
// modes and the tiled set-up passes (shared by both data types).
#include "launch.hpp"
#include "sig_dispatch.hpp"

namespace ffcz {

hipError_t launch_sig_f64(int mode, int lgMc, const void* args, int nsig, hipStream_t s) {
  const SigArgs<double>& a = *static_cast<const SigArgs<double>*>(args);
  switch (mode) {
    case SIG_SETUP: return sig_go<double, double, SIG_SETUP>(lgMc, a, nsig, s);
    case SIG_RUN: return sig_go<double, double, SIG_RUN>(lgMc, a, nsig, s);
    case SIG_RUNL: return sig_go<double, double, SIG_RUNL>(lgMc, a, nsig, s);
    case SIG_VERIFY: return sig_go<double, double, SIG_VERIFY>(lgMc, a, nsig, s);
    case SIGT_CHIRP: return sig_go<double, double, SIGT_CHIRP>(lgMc, a, nsig, s);
    case SIGT_BCOL: return sig_go<double, double, SIGT_BCOL>(lgMc, a, nsig, s);
    case SIGT_BROW: return sig_go<double, double, SIGT_BROW>(lgMc, a, nsig, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
