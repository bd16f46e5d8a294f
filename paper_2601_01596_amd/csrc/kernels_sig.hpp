// One-dimensional signals of any length, one block per signal, the whole
// alternating projection inside one launch.
//
// A real signal of length L is transformed as a complex sequence (imaginary
// part zero); its length-L DFT runs on a power-of-two buffer of Mc = MA*MB
// complex entries in global memory (L2-resident for the lengths of interest):
//   four-step forward: column pass (MB-point FFT over n2 of x[n1 + MA n2],
//     times W_Mc^{n1 k2}), row pass (MA-point FFT over n1); entry (k2, k1)
//     then holds X[k2 + MB k1];
//   four-step inverse: row pass (MA-point inverse, times W_Mc^{-n1 k2}),
//     column pass (MB-point inverse) back to natural order.
// L a power of two: Mc = L and the DFT is the four-step itself.  Otherwise
// Bluestein (chirp z): with w[n] = exp(-i pi n^2 / L) (even in n),
//   X[k] = w[k] (a conv b)[k],  a[n] = v[n] w[n],  b[m] = conj(w[m]),
// the circular convolution done as forward four-step, product with the
// precomputed spectrum of b (times 1/Mc), inverse four-step.  The data are
// real, so only X[k] for k < K = floor(L/2) + 1 is needed, and b only over
// m in [-(L-1), K-1]; the inverse takes only those K coefficients: with
// g[0] = 1, g[L/2] = 1 (L even) and g[k] = 2 otherwise,
//   L eps[n] = Re(U[n]),  U[n] = sum_{k<K} g[k] X'[k] exp(+2 pi i n k / L),
// and conj(U[n]) = w[n] (a2 conv b)[n] with a2[k] = conj(g[k] X'[k]) w[k],
// now over m = n - k in [-(K-1), L-1]: the reflection of the forward range, so
// its spectrum is the forward one at index -k (a second table).  Neither
// range wraps onto itself for Mc >= L + K - 1 (about 1.5 L, against 2L - 1
// for the whole spectrum), which halves Mc for L up to 4/3 of a power of two.
//
// Per round (Alg. 1) the block runs: [row] [column: finish the forward DFT,
// count violations over k <= L/2, clip Re/Im, start the inverse DFT] [row]
// [column: finish the inverse DFT, 1/L, real part, spatial clip, start the
// next forward DFT]; a power-of-two L needs only [row: forward, count, clip,
// inverse] [column: inverse, clip, forward].
//
// Signals whose work buffer fits in LDS (FP32 up to Mc = 2^14, FP64 up to 2^13) keep it
// there for the whole loop (SIG_RUNL): the buffer is stored with a row pitch of MA + 1 and
// every pass exchanges its FFT stages in place inside the tile it owns, so only the tables,
// the iterate and the input and output touch memory.
//
// Long signals run the same passes tiled: each SIGT_* launch does one pass,
// one block per (signal, column tile) or (signal, row tile), and writes one
// partial count per block; sig_ctl_kernel sums them per signal and sets the
// signal's done-flag, which every round pass checks at entry.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "kernels_row.hpp"

namespace ffcz {

struct SigDesc {
  const void* x;      // original (dtype)
  const void* xb;     // base reconstruction (dtype)
  void* y;            // output (dtype)
  int64_t L;
  int32_t blue;       // 1: Bluestein, 0: L == Mc
  int32_t pad;
  double E, Delta, Ep, Dc, Dp;  // bounds, shrunk s-bound, check threshold, shrunk f-bound
  void* conv;         // Mc complex of the working type (aliases conv64)
  void* conv64;       // Mc complex FP64 (set-up and verification)
  void* btab;         // Mc complex, working type, row-pass layout (Bluestein): spectrum of b / Mc
  void* btab64;       // Mc complex FP64, row-pass layout (Bluestein)
  void* btabi;        // Mc complex, working type, row-pass layout: entry k holds entry -k of btab
  void* chirp;        // L complex, working type (Bluestein)
  void* chirp64;      // L complex FP64 (Bluestein)
  void* eps;          // L reals, working type (the iterate)
};

struct SigStats {
  int32_t rounds, converged, nonfinite_stop, done;
  unsigned long long viol0, violf, s_clipped, s_guard, nonfinite, spectral_viol;
  double max_spatial, max_spectral;
};

template <typename T>
struct SigTabs {
  const cx<T>* tw4;   // W_Mc^{n1 k2} at [k2][n1]       (column-pass layout)
  const cx<T>* tw4r;  // W_Mc^{n1 k2} in row-pass layout
  const cx<T>* twa;   // stage twiddles of the MA-point FFT
  const cx<T>* twb;   // stage twiddles of the MB-point FFT
};

template <typename T>
struct SigArgs {
  const SigDesc* sig;
  SigStats* stats;
  const int32_t* order;  // signal index of each block (largest first)
  int32_t nsig;
  int32_t max_iter, fixed, pad;
  SigTabs<T> tab;
  // tiled passes: partial slots [kind][signal slot][tile], kind = SigPart
  unsigned long long* part;
  int32_t ptiles;  // tiles per signal slot in part
  int32_t pad2;
};

enum SigPart : int { SP_VIOL = 0, SP_SCLIP = 1, SP_NONFIN = 2, SP_VMAXF = 3, SP_VCNT = 4, SP_VMAXS = 5, SP_KINDS = 6 };

__host__ __device__ constexpr int imin3(int a, int b, int c) { return a < b ? (a < c ? a : c) : (b < c ? b : c); }
__host__ __device__ constexpr int imax2(int a, int b) { return a > b ? a : b; }

template <typename T, int MA, int MB>
struct SigGeom {
  static constexpr int Mc = MA * MB;
  static constexpr int MB_ = MB;
  static constexpr int EA = pick_E(MA), EB = pick_E(MB);
  static constexpr int PA = MA / EA, PB = MB / EB;
  static constexpr int NTMAX = 512;
  static constexpr int NT = imin3(NTMAX, MA * PB, MB * PA);
  static constexpr int CC = NT / PB;  // columns per column tile
  static constexpr int RR = NT / PA;  // rows per row tile
  static constexpr int LPA = MA + 1;  // LDS pitch of a row (odd)
  static constexpr int LDS = imax2(CC * MB, RR * LPA);
  static constexpr int NCT = MA / CC;  // column tiles (also the element chunks of the tiled passes)
  static constexpr int NRT = MB / RR;  // row tiles
  // the whole work buffer at a row pitch of LPA in one block's LDS (160 KiB per CU, some
  // left for the reductions)
  static constexpr bool RES_FITS = (int64_t)MB * LPA * (int64_t)sizeof(cx<T>) <= 158 * 1024;
  // row-pass table layout: entry (k2, k1) at ((k2 / RR) * MA + k1) * RR + k2 % RR
  __host__ __device__ static constexpr int64_t rpos(int k2, int k1) {
    return ((int64_t)(k2 / RR) * MA + k1) * RR + (k2 % RR);
  }
};

enum SigMode : int {
  // one block per signal, the whole job in one launch
  SIG_SETUP = 0,    // chirp and the spectrum of its conjugate (Bluestein), FP64
  SIG_RUN = 1,      // eps0, every round, y
  SIG_VERIFY = 2,   // FP64 DFT of y - x: maxima and violation count
  // tiled: one pass per launch, one block per (signal, tile)
  SIGT_CHIRP = 3,   // chirp tables, element chunks                          [Bluestein]
  SIGT_BCOL = 4,    // column pass of the conjugate chirp                      [Bluestein]
  SIGT_BROW = 5,    // row pass, store its spectrum / Mc                       [Bluestein]
  SIGT_EPS0 = 6,    // eps0 = x_hat - x (FP64), guard clip; guard and non-finite partials
  SIGT_CIN = 7,     // column pass starting the forward DFT of eps (x chirp)
  SIGT_RMUL = 8,    // row pass: forward, x spectrum of b, inverse            [Bluestein]
  SIGT_RCHECK = 9,  // row pass: forward DFT completes, count, clip, inverse  [power of two]
  SIGT_CCHECK = 10, // column pass: X = w c, count, clip, start the inverse DFT [Bluestein]
  SIGT_CSPAT = 11,  // column pass: finish the inverse DFT, s-clip, next forward start
  SIGT_Y = 12,      // y = x + eps (FP64, clamp); max |y - x| partial
  SIGT_VCOL = 13,   // verification: column pass of d = y - x (FP64)
  SIGT_VROW = 14,   // verification: row pass (Bluestein: x spectrum of b; else maxima partials)
  SIGT_VCOL2 = 15,  // verification: final column pass, maxima partials         [Bluestein]
  SIG_RUNL = 16,    // as SIG_RUN with the work buffer resident in LDS
  SIGT_RMULI = 17   // row pass of the inverse DFT: forward, x reflected spectrum, inverse [Bluestein]
};

__host__ __device__ constexpr bool sig_tiled(int m) { return (m >= SIGT_CHIRP && m <= SIGT_VCOL2) || m == SIGT_RMULI; }
// tiled passes laid out over row tiles; all others over column tiles / element chunks
__host__ __device__ constexpr bool sig_row_tiled(int m) {
  return m == SIGT_BROW || m == SIGT_RMUL || m == SIGT_RMULI || m == SIGT_RCHECK || m == SIGT_VROW;
}
// tiled passes that work on element chunks only (no transform, no LDS)
__host__ __device__ constexpr bool sig_elem_tiled(int m) {
  return m == SIGT_CHIRP || m == SIGT_EPS0 || m == SIGT_Y;
}
// LDS entries a mode needs: a tiled launch runs one kind of pass, so it holds only
// that pass's tile (a column tile of an FP64 2^19 class is half a row tile), which
// lets more blocks share a compute unit
template <typename G, int MODE>
__host__ __device__ constexpr int sig_lds_entries() {
  if constexpr (MODE == SIG_RUNL) return G::MB_ * G::LPA;
  else if constexpr (!sig_tiled(MODE)) return G::LDS;
  else if constexpr (sig_row_tiled(MODE)) return G::RR * G::LPA;
  else if constexpr (sig_elem_tiled(MODE)) return 1;
  else return G::CC * G::MB_;
}

// Block-wide sum / max, result broadcast to every lane.
template <int NT>
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long* red) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_sum_u64(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long s = 0;
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_max_f64(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NW; ++w) s = fmax(s, red[w]);
  return s;
}

template <typename T, typename TIO, int MA, int MB, int MODE>
__global__ void __launch_bounds__((SigGeom<T, MA, MB>::NT))
sig_kernel(SigArgs<T> a) {
  using G = SigGeom<T, MA, MB>;
  constexpr int NT = G::NT, CC = G::CC, RR = G::RR;
  constexpr int EA = G::EA, EB = G::EB, PA = G::PA, PB = G::PB;
  constexpr int LPA = G::LPA;
  constexpr int Mc = MA * MB;
  constexpr int BL = 8;
  __shared__ cx<T> lds[sig_lds_entries<G, MODE>()];
  __shared__ unsigned long long red_u[NT / 64 + 1];
  __shared__ double red_d[NT / 64 + 1];

  constexpr bool tiled = sig_tiled(MODE);
  constexpr int NTL = sig_row_tiled(MODE) ? G::NRT : G::NCT;  // tiles per signal in this launch
  const int slot = tiled ? (int)blockIdx.x / NTL : (int)blockIdx.x;
  const int tile = tiled ? (int)blockIdx.x - slot * NTL : 0;
  if (slot >= a.nsig) return;
  const int sid = a.order ? a.order[slot] : slot;
  const SigDesc sd = a.sig[sid];
  SigStats* so = a.stats + sid;
  const int64_t L = sd.L;
  const bool blue = sd.blue != 0;
  const int t = threadIdx.x;
  // the loop (SIG_RUN and the round passes) works in T = the data type; set-up and
  // verification in FP64 on the FP64 buffers
  constexpr bool loopT = (MODE == SIG_RUN || MODE == SIG_RUNL || MODE == SIGT_EPS0 || MODE == SIGT_CIN ||
                          MODE == SIGT_RMUL || MODE == SIGT_RMULI ||
                          MODE == SIGT_RCHECK || MODE == SIGT_CCHECK || MODE == SIGT_CSPAT || MODE == SIGT_Y);
  // the work buffer: in memory at a row pitch of MA, or (SIG_RUNL) in LDS at a pitch of LPA,
  // where each pass's FFT exchanges run in place inside the tile the pass owns
  constexpr bool RES = MODE == SIG_RUNL;
  constexpr int CP = RES ? LPA : MA;
  cx<T>* conv = RES ? lds : (cx<T>*)(loopT ? sd.conv : sd.conv64);
  const cx<T>* chirp = (const cx<T>*)(loopT ? sd.chirp : sd.chirp64);
  const cx<T>* btab = (const cx<T>*)(loopT ? sd.btab : sd.btab64);
  const cx<T>* btabi = (const cx<T>*)sd.btabi;  // the loop's inverse row passes only
  // tiled partial slot of this block
  auto pslot = [&](int kind) -> unsigned long long& {
    return a.part[((int64_t)kind * a.nsig + slot) * a.ptiles + tile];
  };
  // the tiled round passes stop once the signal's loop has ended
  if constexpr (MODE == SIGT_RMUL || MODE == SIGT_RMULI || MODE == SIGT_RCHECK || MODE == SIGT_CCHECK ||
                MODE == SIGT_CSPAT) {
    if (*(volatile int32_t*)&so->done) return;
  }
  // passes that exist only for one kind of length
  if constexpr (MODE == SIGT_CHIRP || MODE == SIGT_BCOL || MODE == SIGT_BROW || MODE == SIGT_RMUL ||
                MODE == SIGT_RMULI || MODE == SIGT_CCHECK || MODE == SIGT_VCOL2) {
    if (!blue) return;
  }
  if constexpr (MODE == SIGT_RCHECK) {
    if (blue) return;
  }
  // element chunk of the tiled element-wise passes
  constexpr int64_t CH = (int64_t)Mc / G::NCT;
  const int64_t n_lo = tiled ? (int64_t)tile * CH : 0;
  const int64_t n_hi = tiled ? (n_lo + CH < L ? n_lo + CH : L) : L;
  T* eps = (T*)sd.eps;
  const TIO* xs = (const TIO*)sd.x;
  const TIO* xbs = (const TIO*)sd.xb;
  TIO* ys = (TIO*)sd.y;
  const SigTabs<T> tb = a.tab;

  // ---- column pass: for every column n1, inverse MB-FFT (if INV1), element op at the
  // natural index n = n1 + MA*i (or at k2 = i), forward MB-FFT (if FWD2), times the
  // four-step twiddle, store.  in(n1, i) supplies the input when there is no INV1.
  // tiles [tlo, thi) of the pass (all of them in the one-block modes)
  const int ctlo = tiled ? tile : 0, cthi = tiled ? tile + 1 : G::NCT;
  const int rtlo = tiled ? tile : 0, rthi = tiled ? tile + 1 : G::NRT;
  auto col_pass = [&](auto INV1c, auto FWD2c, auto in, auto op) {
    constexpr bool INV1 = decltype(INV1c)::value;
    constexpr bool FWD2 = decltype(FWD2c)::value;
    const int c = t % CC, j = t / CC;
    for (int c0 = ctlo * CC; c0 < cthi * CC; c0 += CC) {
      const int n1 = c0 + c;
      cx<T> v[EB];
      if constexpr (INV1) {
#pragma unroll
        for (int q = 0; q < EB; ++q) v[q] = conv[(int64_t)(j + q * PB) * CP + n1];
        if constexpr (RES) fft<T, MB, EB, true, CP, 1>(v, conv + c0, tb.twb, c, j);
        else fft<T, MB, EB, true, CC, 1>(v, lds, tb.twb, c, j);
      } else {
#pragma unroll
        for (int q = 0; q < EB; ++q) v[q] = in(n1, j + q * PB);
      }
#pragma unroll
      for (int q = 0; q < EB; ++q) v[q] = op(n1, j + q * PB, v[q]);
      if constexpr (FWD2) {
        if constexpr (RES) {
          fft<T, MB, EB, false, CP, 1>(v, conv + c0, tb.twb, c, j);
          __syncthreads();  // the last exchange's reads are done before the tile is overwritten
        } else {
          fft<T, MB, EB, false, CC, 1>(v, lds, tb.twb, c, j);
        }
#pragma unroll
        for (int q = 0; q < EB; ++q) {
          const int64_t p = (int64_t)(j + q * PB) * MA + n1;
          conv[(int64_t)(j + q * PB) * CP + n1] = cmul(v[q], tb.tw4[p]);
        }
      }
    }
    __syncthreads();
  };

  // ---- row pass: for every row k2, forward MA-FFT, element op at (k2, k1), and (if INV)
  // inverse MA-FFT times conj(W_Mc^{n1 k2}); coalesced through LDS in both directions.
  auto row_pass = [&](auto INVc, auto op) {
    constexpr bool INV = decltype(INVc)::value;
    const int rl = t % RR, j = t / RR;
    for (int r0 = rtlo * RR; r0 < rthi * RR; r0 += RR) {
      const int k2 = r0 + rl;
      cx<T> v[EA];
      if constexpr (RES) {
        // the rows are already in LDS at pitch LPA: transform them in place
        cx<T>* rows = conv + (int64_t)r0 * CP;
#pragma unroll
        for (int q = 0; q < EA; ++q) v[q] = rows[rl * CP + j + q * PA];
        fft<T, MA, EA, false, 1, CP>(v, rows, tb.twa, rl, j);
#pragma unroll
        for (int q = 0; q < EA; ++q) v[q] = op(k2, j + q * PA, v[q]);
        if constexpr (INV) {
          fft<T, MA, EA, true, 1, CP>(v, rows, tb.twa, rl, j);
#pragma unroll
          for (int q = 0; q < EA; ++q) v[q] = cmulc(v[q], tb.tw4r[G::rpos(k2, j + q * PA)]);
          __syncthreads();  // the last exchange's reads are done before the rows are overwritten
#pragma unroll
          for (int q = 0; q < EA; ++q) rows[rl * CP + j + q * PA] = v[q];
        }
        __syncthreads();
        continue;
      }
      cx<T>* lrow = lds + rl * LPA;
      constexpr int NL = (RR * MA + NT - 1) / NT;
      // FP64 staging defines every entry on every path (zero where a ragged tile ends),
      // or the batch lands in scratch memory, and a tile of whole block-wide steps
      // (t < NT) drops the per-lane guard.  FP32 keeps the guarded loads (fewer
      // registers live).
      constexpr bool f64 = sizeof(T) == 8;
      constexpr bool whole = f64 && NL * NT == RR * MA;
#pragma unroll
      for (int b0 = 0; b0 < NL; b0 += BL) {
        cx<T> tmp[BL];
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          if constexpr (f64) {
            tmp[u] = (b0 + u < NL && (whole || f < RR * MA)) ? conv[(int64_t)r0 * MA + f] : cx<T>{T(0), T(0)};
          } else if (b0 + u < NL && f < RR * MA) {
            tmp[u] = conv[(int64_t)r0 * MA + f];
          }
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          if (b0 + u < NL && (whole || f < RR * MA)) lds[(f / MA) * LPA + (f % MA)] = tmp[u];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < EA; ++q) v[q] = lrow[j + q * PA];
      fft<T, MA, EA, false, 1, LPA>(v, lds, tb.twa, rl, j);
#pragma unroll
      for (int q = 0; q < EA; ++q) v[q] = op(k2, j + q * PA, v[q]);
      if constexpr (INV) {
        fft<T, MA, EA, true, 1, LPA>(v, lds, tb.twa, rl, j);
#pragma unroll
        for (int q = 0; q < EA; ++q) v[q] = cmulc(v[q], tb.tw4r[G::rpos(k2, j + q * PA)]);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EA; ++q) lrow[j + q * PA] = v[q];
        __syncthreads();
#pragma unroll
        for (int b0 = 0; b0 < NL; b0 += BL) {
#pragma unroll
          for (int u = 0; u < BL; ++u) {
            const int f = t + (b0 + u) * NT;
            if (b0 + u < NL && f < RR * MA) conv[(int64_t)r0 * MA + f] = lds[(f / MA) * LPA + (f % MA)];
          }
        }
      }
      __syncthreads();
    }
  };

  using TT = std::integral_constant<bool, true>;
  using FF = std::integral_constant<bool, false>;
  const cx<T> zero{T(0), T(0)};

  // block-wide partial of a tiled pass
  auto put_sum = [&](int kind, unsigned long long v) {
    v = block_sum<NT>(v, red_u);
    if (t == 0) pslot(kind) = v;
  };
  auto put_max = [&](int kind, double v) {
    v = block_max<NT>(v, red_d);
    if (t == 0) pslot(kind) = (unsigned long long)__double_as_longlong(v);
  };

  if constexpr (MODE == SIG_SETUP || MODE == SIGT_CHIRP || MODE == SIGT_BCOL || MODE == SIGT_BROW) {
    // chirp w[n] = exp(-i pi (n^2 mod 2L) / L) in FP64, and the spectrum of b = conj(w) wrapped
    if (!blue) return;
    // FP32 copies only when the working tables are separate (FP32 batches)
    cx<float>* ch32 = (sd.chirp != sd.chirp64) ? (cx<float>*)sd.chirp : nullptr;
    cx<double>* ch64 = (cx<double>*)sd.chirp64;
    if constexpr (MODE == SIG_SETUP || MODE == SIGT_CHIRP) {
      for (int64_t n = n_lo + t; n < n_hi; n += NT) {
        const int64_t r = (int64_t)(((unsigned long long)n * (unsigned long long)n) % (unsigned long long)(2 * L));
        double s, c;
        sincospi(-(double)r / (double)L, &s, &c);
        ch64[n] = cx<double>{c, s};
        if (ch32) ch32[n] = cx<float>{__double2float_rn(c), __double2float_rn(s)};
      }
      if constexpr (MODE == SIGT_CHIRP) return;
      __syncthreads();
    }
    if constexpr (MODE == SIG_SETUP || MODE == SIGT_BCOL) {
      const int64_t K = L / 2 + 1;
      auto bin = [&](int n1, int i) -> cx<T> {
        const int64_t n = n1 + (int64_t)MA * i;
        int64_t m = -1;
        if (n < K) m = n;                   // b[m], m in [0, K-1]
        else if (n > Mc - L) m = Mc - n;    // b[-m], m in [1, L-1]
        if (m < 0) return zero;
        const cx<double> w = ch64[m];
        return cx<T>{(T)w.re, (T)(-w.im)};
      };
      auto ident = [&](int, int, cx<T> v) { return v; };
      col_pass(FF{}, TT{}, bin, ident);
      if constexpr (MODE == SIGT_BCOL) return;
    }
    // row FFT; store (1/Mc) * spectrum in the row-pass layout of both precisions, and the loop's
    // reflected table: entry k of the spectrum also at index -k (the loop's working type)
    cx<float>* bt32 = (sd.btab != sd.btab64) ? (cx<float>*)sd.btab : nullptr;
    cx<double>* bt64 = (cx<double>*)sd.btab64;
    const double inv = 1.0 / (double)Mc;
    auto store_b = [&](int k2, int k1, cx<T> v) {
      const cx<double> b64{(double)v.re * inv, (double)v.im * inv};
      const cx<float> b32{__double2float_rn(b64.re), __double2float_rn(b64.im)};
      bt64[G::rpos(k2, k1)] = b64;
      if (bt32) bt32[G::rpos(k2, k1)] = b32;  // the row layout does not depend on the type
      const int64_t kr = ((int64_t)Mc - (k2 + (int64_t)MB * k1)) & (Mc - 1);
      const int64_t ri = G::rpos((int)(kr % MB), (int)(kr / MB));
      if (bt32) ((cx<float>*)sd.btabi)[ri] = b32;
      else ((cx<double>*)sd.btabi)[ri] = b64;
      return v;
    };
    row_pass(FF{}, store_b);
    return;
  }

  if constexpr (MODE == SIG_VERIFY || MODE == SIGT_VCOL || MODE == SIGT_VROW || MODE == SIGT_VCOL2) {
    // FP64 DFT of d = y - x: max |d|, max(|Re|,|Im|) and count above Delta over k <= L/2
    double mf = 0.0;
    unsigned long long nv = 0;
    const double D = sd.Delta;
    auto acc = [&](int64_t k, cx<T> X) {
      if (k <= L / 2) {
        const double m = fmax(fabs((double)X.re), fabs((double)X.im));
        mf = fmax(mf, m);
        nv += (m > D) ? 1 : 0;
      }
    };
    auto ident = [&](int, int, cx<T> v) { return v; };
    auto mulb = [&](int k2, int k1, cx<T> v) { return cmul(v, btab[G::rpos(k2, k1)]); };
    auto fin = [&](int n1, int i, cx<T> c) {
      const int64_t n = n1 + (int64_t)MA * i;
      if (n < L) acc(n, cmul(chirp[n], c));
      return c;
    };
    auto rop = [&](int k2, int k1, cx<T> v) {
      acc(k2 + (int64_t)MB * k1, v);
      return v;
    };
    if constexpr (MODE == SIG_VERIFY || MODE == SIGT_VCOL) {
      auto din = [&](int n1, int i) -> cx<T> {
        const int64_t n = n1 + (int64_t)MA * i;
        if (n >= L) return zero;
        const T d = (T)((double)ys[n] - (double)xs[n]);
        if (!blue) return cx<T>{d, T(0)};
        return scal(chirp[n], d);
      };
      col_pass(FF{}, TT{}, din, ident);
      if constexpr (MODE == SIGT_VCOL) return;
    }
    if constexpr (MODE == SIGT_VROW) {
      if (blue) {
        row_pass(TT{}, mulb);
      } else {
        row_pass(FF{}, rop);
        put_max(SP_VMAXF, mf);
        put_sum(SP_VCNT, nv);
      }
      return;
    }
    if constexpr (MODE == SIGT_VCOL2) {
      col_pass(TT{}, FF{}, [&](int, int) { return zero; }, fin);
      put_max(SP_VMAXF, mf);
      put_sum(SP_VCNT, nv);
      return;
    }
    if constexpr (MODE == SIG_VERIFY) {
      double ms = 0.0;
      for (int64_t n = t; n < L; n += NT) ms = fmax(ms, fabs((double)ys[n] - (double)xs[n]));
      ms = block_max<NT>(ms, red_d);
      if (!blue) {
        row_pass(FF{}, rop);
      } else {
        row_pass(TT{}, mulb);
        col_pass(TT{}, FF{}, [&](int, int) { return zero; }, fin);
      }
      mf = block_max<NT>(mf, red_d);
      nv = block_sum<NT>(nv, red_u);
      if (t == 0) {
        so->max_spatial = ms;
        so->max_spectral = mf;
        so->spectral_viol = nv;
      }
      return;
    }
  }

  // ------------------------------------------------------------------ the loop
  const double Ep64 = sd.Ep;
  const T Ep = to_t<T>(sd.Ep);
  const T D = to_t<T>(sd.Dc);
  const T Dp = to_t<T>(sd.Dp);
  const T invL = T(1) / (T)L;
  auto ein = [&](int n1, int i) -> cx<T> {  // a = eps (times the chirp)
    const int64_t n = n1 + (int64_t)MA * i;
    if (n >= L) return zero;
    const T e = eps[n];
    return blue ? scal(chirp[n], e) : cx<T>{e, T(0)};
  };
  auto ident = [&](int, int, cx<T> v) { return v; };
  auto mulb = [&](int k2, int k1, cx<T> v) { return cmul(v, btab[(int64_t)G::rpos(k2, k1)]); };
  auto mulbi = [&](int k2, int k1, cx<T> v) { return cmul(v, btabi[(int64_t)G::rpos(k2, k1)]); };
  const int64_t Kh = L / 2 + 1;  // half-spectrum entries
  unsigned long long cnt = 0, sc = 0;
  // row: the forward DFT completes here -> count + clip -> inverse row FFT (power of two)
  auto rop = [&](int k2, int k1, cx<T> X) {
    const int64_t kk = k2 + (int64_t)MB * k1;
    if (kk <= L / 2 && (fabs(X.re) > D || fabs(X.im) > D)) ++cnt;
    return cx<T>{clipv(X.re, Dp), clipv(X.im, Dp)};
  };
  // column: X = w c for k < K -> count + clip -> start the inverse DFT with conj(g X') w
  // (Bluestein; the entries k >= K are not needed and start the inverse as zero)
  auto fop = [&](int n1, int i, cx<T> c) -> cx<T> {
    const int64_t n = n1 + (int64_t)MA * i;
    if (n >= Kh) return zero;
    const cx<T> w = chirp[n];
    const cx<T> X = cmul(w, c);
    if (fabs(X.re) > D || fabs(X.im) > D) ++cnt;
    const T g = (n == 0 || 2 * n == L) ? T(1) : T(2);
    const cx<T> Xc{g * clipv(X.re, Dp), -(g * clipv(X.im, Dp))};
    return cmul(Xc, w);
  };
  // column: finish the inverse DFT, spatial clip, start the next forward DFT
  auto sop = [&](int n1, int i, cx<T> c) -> cx<T> {
    const int64_t n = n1 + (int64_t)MA * i;
    if (n >= L) return zero;
    T e;
    if (blue) {
      const cx<T> w = chirp[n];
      e = (w.re * c.re - w.im * c.im) * invL;  // Re(conj(w c)) / L
    } else {
      e = c.re * invL;
    }
    if (fabs(e) > Ep) ++sc;
    e = clipv(e, Ep);
    eps[n] = e;
    return blue ? scal(chirp[n], e) : cx<T>{e, T(0)};
  };
  const double Eb = sd.E;

  if constexpr (MODE == SIGT_EPS0 || MODE == SIG_RUN || MODE == SIG_RUNL) {
    // eps0 = x_hat - x in FP64, guard clip
    unsigned long long guard = 0, nonfin = 0;
    for (int64_t n = n_lo + t; n < n_hi; n += NT) {
      double e = (double)xbs[n] - (double)xs[n];
      if (!isfinite(e)) {
        ++nonfin;
        e = 0.0;
      }
      guard += (fabs(e) > Ep64) ? 1 : 0;
      eps[n] = (T)clipv(e, Ep64);
    }
    if constexpr (MODE == SIGT_EPS0) {
      put_sum(SP_SCLIP, guard);
      put_sum(SP_NONFIN, nonfin);
      return;
    }
    if constexpr (MODE == SIG_RUN || MODE == SIG_RUNL) {
      guard = block_sum<NT>(guard, red_u);
      nonfin = block_sum<NT>(nonfin, red_u);
      if (nonfin) {
        if (t == 0) {
          so->nonfinite = nonfin;
          so->nonfinite_stop = 1;
          so->rounds = 0;
          so->converged = 0;
        }
        return;
      }
      __syncthreads();
      col_pass(FF{}, TT{}, ein, ident);
      int k = 0;
      unsigned long long v0 = 0, vk = 0, sclip = 0;
      for (;;) {
        cnt = 0;
        if (!blue) {
          row_pass(TT{}, rop);
        } else {
          row_pass(TT{}, mulb);
          col_pass(TT{}, TT{}, [&](int, int) { return zero; }, fop);
        }
        cnt = block_sum<NT>(cnt, red_u);
        if (k == 0) v0 = cnt;
        vk = cnt;
        if ((!a.fixed && cnt == 0) || k >= a.max_iter) break;
        if (blue) row_pass(TT{}, mulbi);
        sc = 0;
        col_pass(TT{}, TT{}, [&](int, int) { return zero; }, sop);
        sclip += block_sum<NT>(sc, red_u);
        ++k;
      }
      __syncthreads();
      // y = x + eps in FP64, rounded once, closing clamp
      for (int64_t n = t; n < L; n += NT)
        ys[n] = closing_clamp<TIO>(round_io<TIO>((double)xs[n] + (double)eps[n]), xs[n], Eb);
      if (t == 0) {
        so->rounds = k;
        so->converged = (vk == 0) ? 1 : 0;
        so->viol0 = v0;
        so->violf = vk;
        so->s_clipped = sclip;
        so->s_guard = guard;
        so->nonfinite = 0;
        so->nonfinite_stop = 0;
      }
      return;
    }
  }
  if constexpr (MODE == SIGT_CIN) {
    col_pass(FF{}, TT{}, ein, ident);
    return;
  }
  if constexpr (MODE == SIGT_RMUL) {
    row_pass(TT{}, mulb);
    return;
  }
  if constexpr (MODE == SIGT_RMULI) {
    row_pass(TT{}, mulbi);
    return;
  }
  if constexpr (MODE == SIGT_RCHECK) {
    row_pass(TT{}, rop);
    put_sum(SP_VIOL, cnt);
    return;
  }
  if constexpr (MODE == SIGT_CCHECK) {
    col_pass(TT{}, TT{}, [&](int, int) { return zero; }, fop);
    put_sum(SP_VIOL, cnt);
    return;
  }
  if constexpr (MODE == SIGT_CSPAT) {
    col_pass(TT{}, TT{}, [&](int, int) { return zero; }, sop);
    put_sum(SP_SCLIP, sc);
    return;
  }
  if constexpr (MODE == SIGT_Y) {
    double ms = 0.0;
    for (int64_t n = n_lo + t; n < n_hi; n += NT) {
      const TIO yv = closing_clamp<TIO>(round_io<TIO>((double)xs[n] + (double)eps[n]), xs[n], Eb);
      ys[n] = yv;
      ms = fmax(ms, fabs((double)yv - (double)xs[n]));
    }
    put_max(SP_VMAXS, ms);
    return;
  }
}

}  // namespace ffcz
