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
// Bluestein (chirp z): with w[n] = exp(-i pi n^2 / L),
//   X[k] = w[k] (a conv b)[k],  a[n] = v[n] w[n],  b[m] = conj(w[m]) (m in (-L, L)),
// the circular convolution done as forward four-step, product with the
// precomputed spectrum of b (times 1/Mc), inverse four-step, with
// Mc >= 2L - 1.  The inverse DFT is conj(DFT(conj X)).
//
// Per round (Alg. 1) the block runs: [row] [column: finish the forward DFT,
// count violations over k <= L/2, clip Re/Im, start the inverse DFT] [row]
// [column: finish the inverse DFT, 1/L, real part, spatial clip, start the
// next forward DFT]; a power-of-two L needs only [row: forward, count, clip,
// inverse] [column: inverse, clip, forward].
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
  double E, Delta, Ep, Dp;
  void* conv;         // Mc complex of the working type (aliases conv64)
  void* conv64;       // Mc complex FP64 (set-up and verification)
  void* btab;         // Mc complex, working type, row-pass layout (Bluestein)
  void* btab64;       // Mc complex FP64, row-pass layout (Bluestein)
  void* chirp;        // L complex, working type (Bluestein)
  void* chirp64;      // L complex FP64 (Bluestein)
  void* eps;          // L reals, working type (the iterate)
};

struct SigStats {
  int32_t rounds, converged, nonfinite_stop, pad;
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
};

__host__ __device__ constexpr int imin3(int a, int b, int c) { return a < b ? (a < c ? a : c) : (b < c ? b : c); }
__host__ __device__ constexpr int imax2(int a, int b) { return a > b ? a : b; }

template <typename T, int MA, int MB>
struct SigGeom {
  static constexpr int Mc = MA * MB;
  static constexpr int EA = pick_E(MA), EB = pick_E(MB);
  static constexpr int PA = MA / EA, PB = MB / EB;
  static constexpr int NTMAX = 512;
  static constexpr int NT = imin3(NTMAX, MA * PB, MB * PA);
  static constexpr int CC = NT / PB;  // columns per column tile
  static constexpr int RR = NT / PA;  // rows per row tile
  static constexpr int LPA = MA + 1;  // LDS pitch of a row (odd)
  static constexpr int LDS = imax2(CC * MB, RR * LPA);
  // row-pass table layout: entry (k2, k1) at ((k2 / RR) * MA + k1) * RR + k2 % RR
  __host__ __device__ static constexpr int64_t rpos(int k2, int k1) {
    return ((int64_t)(k2 / RR) * MA + k1) * RR + (k2 % RR);
  }
};

enum SigMode : int { SIG_SETUP = 0, SIG_RUN = 1, SIG_VERIFY = 2 };

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
  __shared__ cx<T> lds[G::LDS];
  __shared__ unsigned long long red_u[NT / 64 + 1];
  __shared__ double red_d[NT / 64 + 1];

  if ((int)blockIdx.x >= a.nsig) return;
  const int sid = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  const SigDesc sd = a.sig[sid];
  SigStats* so = a.stats + sid;
  const int64_t L = sd.L;
  const bool blue = sd.blue != 0;
  const int t = threadIdx.x;
  cx<T>* conv = (cx<T>*)(MODE == SIG_RUN ? sd.conv : sd.conv64);
  const cx<T>* chirp = (const cx<T>*)(MODE == SIG_RUN ? sd.chirp : sd.chirp64);
  const cx<T>* btab = (const cx<T>*)(MODE == SIG_RUN ? sd.btab : sd.btab64);
  T* eps = (T*)sd.eps;
  const TIO* xs = (const TIO*)sd.x;
  const TIO* xbs = (const TIO*)sd.xb;
  TIO* ys = (TIO*)sd.y;
  const SigTabs<T> tb = a.tab;

  // ---- column pass: for every column n1, inverse MB-FFT (if INV1), element op at the
  // natural index n = n1 + MA*i (or at k2 = i), forward MB-FFT (if FWD2), times the
  // four-step twiddle, store.  in(n1, i) supplies the input when there is no INV1.
  auto col_pass = [&](auto INV1c, auto FWD2c, auto in, auto op) {
    constexpr bool INV1 = decltype(INV1c)::value;
    constexpr bool FWD2 = decltype(FWD2c)::value;
    const int c = t % CC, j = t / CC;
    for (int c0 = 0; c0 < MA; c0 += CC) {
      const int n1 = c0 + c;
      cx<T> v[EB];
      if constexpr (INV1) {
#pragma unroll
        for (int q = 0; q < EB; ++q) v[q] = conv[(int64_t)(j + q * PB) * MA + n1];
        fft<T, MB, EB, true, CC, 1>(v, lds, tb.twb, c, j);
      } else {
#pragma unroll
        for (int q = 0; q < EB; ++q) v[q] = in(n1, j + q * PB);
      }
#pragma unroll
      for (int q = 0; q < EB; ++q) v[q] = op(n1, j + q * PB, v[q]);
      if constexpr (FWD2) {
        fft<T, MB, EB, false, CC, 1>(v, lds, tb.twb, c, j);
#pragma unroll
        for (int q = 0; q < EB; ++q) {
          const int64_t p = (int64_t)(j + q * PB) * MA + n1;
          conv[p] = cmul(v[q], tb.tw4[p]);
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
    cx<T>* lrow = lds + rl * LPA;
    for (int r0 = 0; r0 < MB; r0 += RR) {
      constexpr int NL = (RR * MA + NT - 1) / NT;
#pragma unroll
      for (int b0 = 0; b0 < NL; b0 += BL) {
        cx<T> tmp[BL];
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          if (b0 + u < NL && f < RR * MA) tmp[u] = conv[(int64_t)r0 * MA + f];
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          if (b0 + u < NL && f < RR * MA) lds[(f / MA) * LPA + (f % MA)] = tmp[u];
        }
      }
      __syncthreads();
      cx<T> v[EA];
#pragma unroll
      for (int q = 0; q < EA; ++q) v[q] = lrow[j + q * PA];
      fft<T, MA, EA, false, 1, LPA>(v, lds, tb.twa, rl, j);
      const int k2 = r0 + rl;
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

  if constexpr (MODE == SIG_SETUP) {
    // chirp w[n] = exp(-i pi (n^2 mod 2L) / L) in FP64, and the spectrum of b = conj(w) wrapped
    if (!blue) return;
    // FP32 copies only when the working tables are separate (FP32 batches)
    cx<float>* ch32 = (sd.chirp != sd.chirp64) ? (cx<float>*)sd.chirp : nullptr;
    cx<double>* ch64 = (cx<double>*)sd.chirp64;
    for (int64_t n = t; n < L; n += NT) {
      const int64_t r = (int64_t)(((unsigned long long)n * (unsigned long long)n) % (unsigned long long)(2 * L));
      double s, c;
      sincospi(-(double)r / (double)L, &s, &c);
      ch64[n] = cx<double>{c, s};
      if (ch32) ch32[n] = cx<float>{__double2float_rn(c), __double2float_rn(s)};
    }
    __syncthreads();
    auto bin = [&](int n1, int i) -> cx<T> {
      const int64_t n = n1 + (int64_t)MA * i;
      int64_t m = -1;
      if (n < L) m = n;
      else if (n > Mc - L) m = Mc - n;
      if (m < 0) return zero;
      const cx<double> w = ch64[m];
      return cx<T>{(T)w.re, (T)(-w.im)};
    };
    auto ident = [&](int, int, cx<T> v) { return v; };
    col_pass(FF{}, TT{}, bin, ident);
    // row FFT; store (1/Mc) * spectrum in the row-pass layout of both precisions
    cx<float>* bt32 = (sd.btab != sd.btab64) ? (cx<float>*)sd.btab : nullptr;
    cx<double>* bt64 = (cx<double>*)sd.btab64;
    const double inv = 1.0 / (double)Mc;
    auto store_b = [&](int k2, int k1, cx<T> v) {
      bt64[G::rpos(k2, k1)] = cx<double>{(double)v.re * inv, (double)v.im * inv};
      if (bt32) {
        using G32 = SigGeom<float, MA, MB>;
        bt32[G32::rpos(k2, k1)] = cx<float>{__double2float_rn((double)v.re * inv), __double2float_rn((double)v.im * inv)};
      }
      return v;
    };
    row_pass(FF{}, store_b);
    return;
  }

  if constexpr (MODE == SIG_VERIFY) {
    // FP64 DFT of d = y - x: max |d|, max(|Re|,|Im|) and count above Delta over k <= L/2
    double ms = 0.0;
    for (int64_t n = t; n < L; n += NT) ms = fmax(ms, fabs((double)ys[n] - (double)xs[n]));
    ms = block_max<NT>(ms, red_d);
    auto din = [&](int n1, int i) -> cx<T> {
      const int64_t n = n1 + (int64_t)MA * i;
      if (n >= L) return zero;
      const T d = (T)((double)ys[n] - (double)xs[n]);
      if (!blue) return cx<T>{d, T(0)};
      return scal(chirp[n], d);
    };
    auto ident = [&](int, int, cx<T> v) { return v; };
    col_pass(FF{}, TT{}, din, ident);
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
    if (!blue) {
      auto rop = [&](int k2, int k1, cx<T> v) {
        acc(k2 + (int64_t)MB * k1, v);
        return v;
      };
      row_pass(FF{}, rop);
    } else {
      auto mulb = [&](int k2, int k1, cx<T> v) { return cmul(v, btab[G::rpos(k2, k1)]); };
      row_pass(TT{}, mulb);
      auto fin = [&](int n1, int i, cx<T> c) {
        const int64_t n = n1 + (int64_t)MA * i;
        if (n < L) acc(n, cmul(chirp[n], c));
        return c;
      };
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

  // ------------------------------------------------------------------ SIG_RUN
  const double Ep64 = sd.Ep;
  const T Ep = to_t<T>(sd.Ep);
  const T D = to_t<T>(sd.Delta);
  const T Dp = to_t<T>(sd.Dp);
  const T invL = T(1) / (T)L;
  // eps0 = x_hat - x in FP64, guard clip
  unsigned long long guard = 0, nonfin = 0;
  for (int64_t n = t; n < L; n += NT) {
    double e = (double)xbs[n] - (double)xs[n];
    if (!isfinite(e)) {
      ++nonfin;
      e = 0.0;
    }
    guard += (fabs(e) > Ep64) ? 1 : 0;
    eps[n] = (T)clipv(e, Ep64);
  }
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

  auto ein = [&](int n1, int i) -> cx<T> {  // a = eps (times the chirp)
    const int64_t n = n1 + (int64_t)MA * i;
    if (n >= L) return zero;
    const T e = eps[n];
    return blue ? scal(chirp[n], e) : cx<T>{e, T(0)};
  };
  auto ident = [&](int, int, cx<T> v) { return v; };
  col_pass(FF{}, TT{}, ein, ident);

  int k = 0;
  unsigned long long v0 = 0, vk = 0, sclip = 0;
  for (;;) {
    unsigned long long cnt = 0;
    if (!blue) {
      // row: the forward DFT completes here -> count + clip -> inverse row FFT
      auto rop = [&](int k2, int k1, cx<T> X) {
        const int64_t kk = k2 + (int64_t)MB * k1;
        if (kk <= L / 2 && (fabs(X.re) > D || fabs(X.im) > D)) ++cnt;
        return cx<T>{clipv(X.re, Dp), clipv(X.im, Dp)};
      };
      row_pass(TT{}, rop);
    } else {
      auto mulb = [&](int k2, int k1, cx<T> v) { return cmul(v, btab[(int64_t)G::rpos(k2, k1)]); };
      row_pass(TT{}, mulb);
      // column: X = w c -> count + clip -> start the inverse DFT with conj(X') w
      auto fop = [&](int n1, int i, cx<T> c) -> cx<T> {
        const int64_t n = n1 + (int64_t)MA * i;
        if (n >= L) return zero;
        const cx<T> w = chirp[n];
        const cx<T> X = cmul(w, c);
        if (n <= L / 2 && (fabs(X.re) > D || fabs(X.im) > D)) ++cnt;
        const cx<T> Xc{clipv(X.re, Dp), -clipv(X.im, Dp)};
        return cmul(Xc, w);
      };
      col_pass(TT{}, TT{}, [&](int, int) { return zero; }, fop);
    }
    cnt = block_sum<NT>(cnt, red_u);
    if (k == 0) v0 = cnt;
    vk = cnt;
    if ((!a.fixed && cnt == 0) || k >= a.max_iter) break;
    if (blue) {
      auto mulb = [&](int k2, int k1, cx<T> v) { return cmul(v, btab[(int64_t)G::rpos(k2, k1)]); };
      row_pass(TT{}, mulb);
    }
    // column: finish the inverse DFT, spatial clip, start the next forward DFT
    unsigned long long sc = 0;
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
    col_pass(TT{}, TT{}, [&](int, int) { return zero; }, sop);
    sclip += block_sum<NT>(sc, red_u);
    ++k;
  }
  __syncthreads();
  // y = x + eps in FP64, rounded once, closing clamp
  const double Eb = sd.E;
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
}

}  // namespace ffcz
