// Runtime work length -> templated per-signal kernel.  One-block modes exist
// for every length class; the tiled passes only from kSigTiledMinLg on (shorter
// signals always run one block each).
#pragma once
#include "kernels_sig.hpp"

namespace ffcz {

constexpr int kSigTiledMinLg = 12;

template <typename T, typename TIO, int MODE, int MA, int MB>
hipError_t sig_launch_one(const SigArgs<T>& a, int nsig, hipStream_t s) {
  using G = SigGeom<T, MA, MB>;
  const int per = sig_tiled(MODE) ? (sig_row_tiled(MODE) ? G::NRT : G::NCT) : 1;
  const int64_t nb = (int64_t)nsig * per;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((sig_kernel<T, TIO, MA, MB, MODE>), dim3((unsigned)nb), dim3(G::NT), 0, s, a);
  return hipGetLastError();
}

template <typename T, typename TIO, int MODE>
hipError_t sig_go(int lgMc, const SigArgs<T>& a, int nsig, hipStream_t s) {
  if (sig_tiled(MODE) && lgMc < kSigTiledMinLg) return hipErrorInvalidValue;
  switch (lgMc) {
#define FFCZ_CASE(LG, MA, MB) \
  case LG:                    \
    if constexpr ((!sig_tiled(MODE) || LG >= kSigTiledMinLg) && (MODE != SIG_RUNL || SigGeom<T, MA, MB>::RES_FITS)) \
      return sig_launch_one<T, TIO, MODE, MA, MB>(a, nsig, s);                                                        \
    break;
    FFCZ_CASE(2, 2, 2) FFCZ_CASE(3, 4, 2) FFCZ_CASE(4, 4, 4) FFCZ_CASE(5, 8, 4) FFCZ_CASE(6, 8, 8)
    FFCZ_CASE(7, 16, 8) FFCZ_CASE(8, 16, 16) FFCZ_CASE(9, 32, 16) FFCZ_CASE(10, 32, 32)
    FFCZ_CASE(11, 64, 32) FFCZ_CASE(12, 64, 64) FFCZ_CASE(13, 128, 64) FFCZ_CASE(14, 128, 128)
    FFCZ_CASE(15, 256, 128) FFCZ_CASE(16, 256, 256) FFCZ_CASE(17, 512, 256) FFCZ_CASE(18, 512, 512)
    FFCZ_CASE(19, 1024, 512) FFCZ_CASE(20, 1024, 1024)
#undef FFCZ_CASE
    default: break;
  }
  return hipErrorInvalidValue;
}

// Whether a class's work buffer fits in one block's LDS (SIG_RUNL), mirror of SigGeom::RES_FITS.
inline bool sig_res_fits(int dt, int lgMc) {
  const int64_t MA = (int64_t)1 << ((lgMc + 1) / 2), MB = ((int64_t)1 << lgMc) / MA;
  return MB * (MA + 1) * (dt == 0 ? 8 : 16) <= 158 * 1024;
}

// Tiles per signal of a tiled mode (grid = signals x tiles), for the host's partial buffers.
inline void sig_tiles(int lgMc, int* nct, int* nrt) {
  const int MA = 1 << ((lgMc + 1) / 2), MB = (1 << lgMc) / MA;
  const int PA = MA / pick_E(MA), PB = MB / pick_E(MB);
  const int NT = imin3(512, MA * PB, MB * PA);
  *nct = MA / (NT / PB);
  *nrt = MB / (NT / PA);
}

}  // namespace ffcz
