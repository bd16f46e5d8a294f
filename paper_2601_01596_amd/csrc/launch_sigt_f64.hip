// Dispatch of the tiled per-signal passes computing in double: the FP64 loop
// and the FP64 verification of float or double data.
#include "launch.hpp"
#include "sig_dispatch.hpp"

namespace ffcz {

hipError_t launch_sigt_f64(int mode, int iodt, int lgMc, const void* args, int nsig, hipStream_t s) {
  const SigArgs<double>& a = *static_cast<const SigArgs<double>*>(args);
  if (iodt == 0) {
    switch (mode) {
      case SIGT_VCOL: return sig_go<double, float, SIGT_VCOL>(lgMc, a, nsig, s);
      case SIGT_VROW: return sig_go<double, float, SIGT_VROW>(lgMc, a, nsig, s);
      case SIGT_VCOL2: return sig_go<double, float, SIGT_VCOL2>(lgMc, a, nsig, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (mode) {
    case SIGT_EPS0: return sig_go<double, double, SIGT_EPS0>(lgMc, a, nsig, s);
    case SIGT_CIN: return sig_go<double, double, SIGT_CIN>(lgMc, a, nsig, s);
    case SIGT_RMUL: return sig_go<double, double, SIGT_RMUL>(lgMc, a, nsig, s);
    case SIGT_RMULI: return sig_go<double, double, SIGT_RMULI>(lgMc, a, nsig, s);
    case SIGT_RCHECK: return sig_go<double, double, SIGT_RCHECK>(lgMc, a, nsig, s);
    case SIGT_CCHECK: return sig_go<double, double, SIGT_CCHECK>(lgMc, a, nsig, s);
    case SIGT_CSPAT: return sig_go<double, double, SIGT_CSPAT>(lgMc, a, nsig, s);
    case SIGT_Y: return sig_go<double, double, SIGT_Y>(lgMc, a, nsig, s);
    case SIGT_VCOL: return sig_go<double, double, SIGT_VCOL>(lgMc, a, nsig, s);
    case SIGT_VROW: return sig_go<double, double, SIGT_VROW>(lgMc, a, nsig, s);
    case SIGT_VCOL2: return sig_go<double, double, SIGT_VCOL2>(lgMc, a, nsig, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffcz
