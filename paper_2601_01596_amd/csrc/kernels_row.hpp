// Last-axis passes.  A block owns ROWS rows of the half-spectrum (H+1 complex
// entries each, H = n_last/2) and runs the real transforms through a complex
// transform of length H: the real row r is packed as z[m] = r[2m] + i r[2m+1].
//   C2R:  Z'[k] = (X[k] + X[H-k]*) + i W^-k (X[k] - X[H-k]*),  r = IDFT_H(Z') / n
//   R2C:  X[k] = (Z[k] + Z[H-k]*)/2 - i W^k (Z[k] - Z[H-k]*)/2,  X[H] = Re Z0 - Im Z0
// with W = exp(-2 pi i / n).  The imaginary parts of X[0] and X[H] are taken
// as zero, as a real inverse transform does.  The spatial projection runs on
// the lane's registers between the two transforms, so the spatial error never
// leaves the chip.
#pragma once
#include "common.hpp"

namespace ffcz {

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
  using type = float2;
};
template <>
struct Vec2<double> {
  using type = double2;
};

// Round an FP64 value to TIO (nearest even).
template <typename TIO>
__device__ __forceinline__ TIO round_io(double v);
template <>
__device__ __forceinline__ float round_io<float>(double v) { return __double2float_rn(v); }
template <>
__device__ __forceinline__ double round_io<double>(double v) { return v; }

// Move y one representable step toward x until |y - x| <= E holds in FP64.
template <typename TIO>
__device__ __forceinline__ TIO closing_clamp(TIO y, TIO x, double E) {
  for (int it = 0; it < 64; ++it) {
    if (fabs((double)y - (double)x) <= E) return y;
    y = nextafter(y, x);
  }
  return (fabs((double)y - (double)x) <= E) ? y : x;
}

template <typename T, typename TIO, int H, int ROWS, int MODE>
__global__ void __launch_bounds__(ROWS*(H / pick_E(H)))
row_kernel(RowArgs<T, TIO> a) {
  constexpr int E = pick_E(H);
  constexpr int P = H / E;
  constexpr int NT = ROWS * P;
  constexpr int LP = H + 1;
  using S = Sched<H, E>;
  constexpr int TW = S::twsize;
  constexpr int NW = (NT + 63) / 64;
  constexpr int SW = 2 * (H >= 32 ? H / 32 : 1);  // uint32 words per s-mask row (64-bit padded)
  using V2 = typename Vec2<TIO>::type;

  __shared__ cx<T> lds[ROWS * LP];
  __shared__ cx<T> tws[TW + H];
  __shared__ unsigned long long red_u[NW];
  __shared__ double red_d[NW];
  __shared__ uint32_t sbits[ROWS * SW];

  DevState* st = a.st;
  constexpr bool uses_done = (MODE == ROW_LOOP);
  if (uses_done) {
    if (*(volatile int32_t*)&st->done) return;
  }
  const int t = threadIdx.x;
  const int rl = t / P;
  const int j = t - rl * P;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  const int64_t g = row0 + rl;
  const bool valid = g < a.nrows;
  cx<T>* lrow = lds + rl * LP;
  const cx<T>* rtw = tws + TW;

  for (int i = t; i < TW + H; i += NT) tws[i] = a.tw[i];
  constexpr bool rec_s = (MODE == ROW_INIT || MODE == ROW_LOOP);
  int kround = 0;
  bool rec = false;
  if constexpr (rec_s) {
    if (MODE == ROW_LOOP) kround = *(volatile int32_t*)&st->round;
    rec = st->record_masks != 0;
    if (rec) {
      for (int i = t; i < ROWS * SW; i += NT) sbits[i] = 0u;
      __syncthreads();
    }
  }

  cx<T> v[E];
  unsigned long long cnt = 0;
  double mx = 0.0;

  if constexpr (MODE == ROW_INIT || MODE == ROW_VERIFY || MODE == ROW_BINIT) {
    // real input rows -> packed complex registers
    const V2* x2 = reinterpret_cast<const V2*>(a.x);
    const V2* b2 = reinterpret_cast<const V2*>(a.xb);
    const double Ep = st->Ep;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      double e0 = 0.0, e1 = 0.0;
      if (valid) {
        if constexpr (MODE == ROW_BINIT) {
          const V2 gv = b2[g * H + k];
          e0 = (double)gv.x;
          e1 = (double)gv.y;
          const uint32_t w = a.smask[g * a.s_row_w32 + (2 * k) / 32];
          const int sh = (2 * k) & 31;
          e0 = ((w >> sh) & 1u) ? e0 : 0.0;
          e1 = ((w >> (sh + 1)) & 1u) ? e1 : 0.0;
        } else {
          const V2 xv = x2[g * H + k];
          const V2 bv = b2[g * H + k];
          e0 = (double)bv.x - (double)xv.x;
          e1 = (double)bv.y - (double)xv.y;
          if constexpr (MODE == ROW_INIT) {
            const bool f0 = isfinite(e0), f1 = isfinite(e1);
            if (!f0 || !f1) {
              atomicAdd(&st->nonfinite, (unsigned long long)((!f0) + (!f1)));
              e0 = f0 ? e0 : 0.0;
              e1 = f1 ? e1 : 0.0;
            }
            const bool k0 = fabs(e0) <= Ep, k1 = fabs(e1) <= Ep;
            cnt += (!k0) + (!k1);
            e0 = clipv(e0, Ep);
            e1 = clipv(e1, Ep);
            if (rec) atomicOr(&sbits[rl * SW + (2 * k) / 32], ((uint32_t)k0 | ((uint32_t)k1 << 1)) << ((2 * k) & 31));
          } else {
            mx = fmax(mx, fmax(fabs(e0), fabs(e1)));
          }
        }
      }
      v[q] = cx<T>{(T)e0, (T)e1};  // eps0 is rounded once to the working type
    }
  } else {
    // spectrum row -> LDS -> packed C2R input
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      lrow[k] = valid ? a.src[g * a.pitch + k] : cx<T>{T(0), T(0)};
    }
    if (j == 0) lrow[H] = valid ? a.src[g * a.pitch + H] : cx<T>{T(0), T(0)};
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      cx<T> A = lrow[k];
      cx<T> B = lrow[H - k];
      if (k == 0) {
        A.im = T(0);
        B.im = T(0);
      }
      const cx<T> sm = A + conjg(B);
      const cx<T> df = cmulc(A - conjg(B), rtw[k]);  // W^-k (A - B*)
      v[q] = cx<T>{sm.re - df.im, sm.im + df.re};    // sm + i * df
    }
    fft<T, H, E, true, 1, LP>(v, lds, tws, rl, j);
    const T sc = (T)st->inv_n;
    if constexpr (MODE == ROW_FINAL) {
      // the source holds only the last-axis R2C of eps, so the C2R scale is 1/n_last
      const T scz = T(1) / T(2 * H);
      const V2* x2 = reinterpret_cast<const V2*>(a.x);
      V2* y2 = reinterpret_cast<V2*>(a.y);
      const double Eb = st->E;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int k = j + q * P;
        if (valid) {
          const V2 xv = x2[g * H + k];
          const double e0 = (double)(v[q].re * scz), e1 = (double)(v[q].im * scz);
          TIO y0 = round_io<TIO>((double)xv.x + e0);
          TIO y1 = round_io<TIO>((double)xv.y + e1);
          y0 = closing_clamp<TIO>(y0, xv.x, Eb);
          y1 = closing_clamp<TIO>(y1, xv.y, Eb);
          V2 out;
          out.x = y0;
          out.y = y1;
          y2[g * H + k] = out;
        }
      }
      return;
    } else if constexpr (MODE == ROW_BLOOP || MODE == ROW_BFINAL) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int k = j + q * P;
        uint32_t w = 0;
        if (valid) w = a.smask[g * a.s_row_w32 + (2 * k) / 32];
        const int sh = (2 * k) & 31;
        const T e0 = ((w >> sh) & 1u) ? v[q].re * sc : T(0);
        const T e1 = ((w >> (sh + 1)) & 1u) ? v[q].im * sc : T(0);
        v[q] = cx<T>{e0, e1};
      }
      if constexpr (MODE == ROW_BFINAL) {
        V2* y2 = reinterpret_cast<V2*>(a.y);
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int k = j + q * P;
          if (valid) {
            V2 out;
            out.x = (TIO)v[q].re;
            out.y = (TIO)v[q].im;
            y2[g * H + k] = out;
          }
        }
        return;
      }
    } else {  // ROW_LOOP: ProjectOntoSCube
      const T Ep = to_t<T>(st->Ep);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int k = j + q * P;
        T e0 = v[q].re * sc, e1 = v[q].im * sc;
        const bool k0 = fabs(e0) <= Ep, k1 = fabs(e1) <= Ep;
        if (valid) cnt += (!k0) + (!k1);
        e0 = clipv(e0, Ep);
        e1 = clipv(e1, Ep);
        v[q] = cx<T>{e0, e1};
        if (rec && valid)
          atomicOr(&sbits[rl * SW + (2 * k) / 32], ((uint32_t)k0 | ((uint32_t)k1 << 1)) << ((2 * k) & 31));
      }
    }
  }

  // ---- forward R2C of the packed registers
  fft<T, H, E, false, 1, LP>(v, lds, tws, rl, j);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) lrow[j + q * P] = v[q];
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      const cx<T> Zk = v[q];
      const cx<T> Zm = lrow[(H - k) & (H - 1)];
      const cx<T> ev = scal(Zk + conjg(Zm), T(0.5));
      const cx<T> d = Zk - conjg(Zm);
      const cx<T> od = cx<T>{d.im * T(0.5), -d.re * T(0.5)};  // d / (2i)
      a.dst[g * a.pitch + k] = ev + cmul(rtw[k], od);
    }
    if (j == 0) a.dst[g * a.pitch + H] = cx<T>{v[0].re - v[0].im, T(0)};
  }

  // ---- counters and masks
  if constexpr (MODE == ROW_INIT || MODE == ROW_LOOP || MODE == ROW_VERIFY) {
    cnt = wave_sum_u64(cnt);
    mx = wave_max_f64(mx);
    if ((t & 63) == 0) {
      red_u[t >> 6] = cnt;
      red_d[t >> 6] = mx;
    }
    __syncthreads();
    if (t == 0) {
      unsigned long long s = 0;
      double m = 0.0;
      for (int w = 0; w < NW; ++w) {
        s += red_u[w];
        m = fmax(m, red_d[w]);
      }
      // one partial per block, reduced by the control / statistics kernels
      if constexpr (MODE == ROW_VERIFY) a.part[blockIdx.x] = (unsigned long long)__double_as_longlong(m);
      else a.part[blockIdx.x] = s;
    }
    if constexpr (rec_s) {
      if (rec) {
        uint32_t* plane = a.smask + (int64_t)kround * a.s_plane;
        for (int i = t; i < ROWS * SW; i += NT) {
          const int r = i / SW;
          const int w = i - r * SW;
          if (row0 + r < a.nrows && w < a.s_row_w32) plane[(row0 + r) * a.s_row_w32 + w] = sbits[i];
        }
      }
    }
  }
}

}  // namespace ffcz
