// Register/LDS Stockham FFT engine for gfx950 (power-of-two lengths).
//
// A transform of length L is spread over P = L/E lanes; lane j keeps the E
// elements j + q*P (q = 0..E-1) in registers.  Stages run in Stockham
// (self-sorting) order: a first stage of radix r0 = L / E^a when L is not a
// power of E, then a stages of radix E.  Stage s with span Ns reads the
// butterfly inputs jb + r*L/R (already in the lane's registers), multiplies
// input r by exp(-+2 pi i (jb mod Ns) r / (Ns R)), runs an R-point DFT and
// writes output r to index (jb/Ns)*Ns*R + (jb mod Ns) + r*Ns.  Intermediate
// stages exchange through LDS; the last stage's outputs land back in natural
// order j + q*P in the same registers, so a forward transform, an elementwise
// projection and an inverse transform chain without an extra exchange.
//
// Sign convention: forward = exp(-2 pi i k n / L) (Eq. 1 of the paper),
// inverse = exp(+...), both unnormalised.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffcz {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> scal(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  if constexpr (INV) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// cos and sin of 2 pi k / 16, k = 0..15, as exact-to-double literals.
__host__ __device__ constexpr double cos16(int k) {
  switch (k & 15) {
    case 0: return 1.0;
    case 1: return 0.92387953251128675613;
    case 2: return 0.70710678118654752440;
    case 3: return 0.38268343236508977173;
    case 4: return 0.0;
    case 5: return -0.38268343236508977173;
    case 6: return -0.70710678118654752440;
    case 7: return -0.92387953251128675613;
    case 8: return -1.0;
    case 9: return -0.92387953251128675613;
    case 10: return -0.70710678118654752440;
    case 11: return -0.38268343236508977173;
    case 12: return 0.0;
    case 13: return 0.38268343236508977173;
    case 14: return 0.70710678118654752440;
    default: return 0.92387953251128675613;
  }
}
__host__ __device__ constexpr double sin16(int k) { return cos16(k + 12); }  // sin x = cos(x - pi/2)

// x * W_R^k with W_R = exp(-+2 pi i / R), R | 16; k is a compile-time constant after unrolling.
template <int R, bool INV, typename T>
__device__ __forceinline__ cx<T> twc(cx<T> x, int k) {
  const int k16 = (k * (16 / R)) & 15;
  if (k16 == 0) return x;
  if (k16 == 4) return mul_mi<INV>(x);
  if (k16 == 8) return {-x.re, -x.im};
  if (k16 == 12) return mul_mi<!INV>(x);
  const T c = (T)cos16(k16);
  const T s = INV ? (T)sin16(k16) : (T)(-sin16(k16));
  return {x.re * c - x.im * s, x.re * s + x.im * c};
}

// In-register R-point DFT, natural order in and out (radix-2 decimation in time).
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T> (&v)[R]) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    const cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    const cx<T> s13 = v[1] + v[3], d13 = mul_mi<INV>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
  } else {
    constexpr int H = R / 2;
    cx<T> e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<H, INV>(e);
    dft<H, INV>(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const cx<T> t = twc<R, INV>(o[k], k);
      v[k] = e[k] + t;
      v[k + H] = e[k] - t;
    }
  }
}

__host__ __device__ constexpr int ilog2c(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

// Elements per lane for a length-L transform.
__host__ __device__ constexpr int pick_E(int L) { return L <= 16 ? L : (L <= 512 ? 8 : 16); }

// Stage schedule of a length-L transform with E elements per lane.
template <int L, int E>
struct Sched {
  static constexpr int lgL = ilog2c(L);
  static constexpr int lgE = ilog2c(E);
  static constexpr int a = (E <= 1) ? 0 : lgL / lgE;  // radix-E stages
  static constexpr int r0 = (E <= 1) ? 1 : (L >> (a * lgE));
  static constexpr int nst = a + (r0 > 1 ? 1 : 0);
  static constexpr int radix(int s) { return (r0 > 1 && s == 0) ? r0 : E; }
  static constexpr int ns(int s) {
    int n = 1;
    for (int t = 0; t < s; ++t) n *= radix(t);
    return n;
  }
  // Offset (in complex entries) of stage s's twiddle table; stages with Ns = 1 have none.
  static constexpr int twoff(int s) {
    int o = 0;
    for (int t = 0; t < s; ++t)
      if (ns(t) > 1) o += ns(t) * (radix(t) - 1);
    return o;
  }
  static constexpr int twsize = twoff(nst);
};

// Twiddle-table entries of the stage plan for a runtime length L (the plan Sched
// fixes at compile time): an optional radix-r0 stage at span 1, then radix-E stages
// at spans r0 E^t; a stage of span ns > 1 owns ns (radix - 1) entries, in stage
// order (the span-1 stage owns none).
__host__ __device__ constexpr int host_twsize(int L, int E) {
  if (E <= 1 || L <= 1) return 0;
  const int lgE = ilog2c(E), a = ilog2c(L) / lgE;
  const int r0 = L >> (a * lgE);
  int s = 0, ns = r0 > 1 ? r0 : 1;
  for (int t = 0; t < a; ++t, ns *= E)
    if (ns > 1) s += ns * (E - 1);
  return s;
}

// Element (b, i) of the LDS batch lives at lds[sk(i)*SI + b*SB], with sk(i) = i
// (SK = 0) or i + (i >> SK) (a skip every 2^SK entries, against bank conflicts).
template <int SK>
__device__ __forceinline__ int lds_skew(int i) {
  if constexpr (SK > 0) return i + (i >> SK);
  else return i;
}

// SPL: exchange the real parts, then the imaginary parts, through an LDS area of one real
// per entry (half the footprint, two more barriers per exchange; same arithmetic, same bits).
template <typename T, int L, int E, bool INV, int SI, int SB, int s, int SK = 0, bool SPL = false>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[E], cx<T>* lds, const cx<T>* tw, int b, int j) {
  using S = Sched<L, E>;
  if constexpr (s < S::nst) {
    constexpr int R = S::radix(s);
    constexpr int Ns = S::ns(s);
    constexpr int NB = E / R;
    constexpr int P = L / E;
    constexpr bool last = (s == S::nst - 1);
    cx<T> u[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int jb = j + i * P;
#pragma unroll
      for (int r = 0; r < R; ++r) u[i][r] = v[i + r * NB];
      if constexpr (Ns > 1) {
        const cx<T>* t = tw + S::twoff(s) + (jb & (Ns - 1)) * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) u[i][r] = INV ? cmulc(u[i][r], t[r - 1]) : cmul(u[i][r], t[r - 1]);
      }
      dft<R, INV>(u[i]);
    }
    if constexpr (last) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) v[i + r * NB] = u[i][r];
    } else {
      // slot of element r of lane group i (the write side of the exchange)
      auto wslot = [&](int i, int r) -> int {
        const int jb = j + i * P;
        const int base = (jb / Ns) * (Ns * R) + (jb & (Ns - 1));
        if constexpr (SK > 0 && (Ns * R) % (1 << SK) == 0) {
          // with Ns R a multiple of 2^SK, sk(base + r Ns) = sk-part of base + sk(r Ns):
          // one lane base, compile-time offsets
          const int lb = base + (jb / Ns) * ((Ns * R) >> SK) + ((jb & (Ns - 1)) >> SK);
          return (lb + lds_skew<SK>(r * Ns)) * SI + b * SB;
        } else {
          return lds_skew<SK>(base + r * Ns) * SI + b * SB;
        }
      };
      // j < P and P a power of two: sk(j + qP) = sk(j) + sk(qP), a lane base plus constants
      const int sj = lds_skew<SK>(j);
      if constexpr (SPL) {
        T* lr = reinterpret_cast<T*>(lds);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          __syncthreads();
#pragma unroll
          for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) lr[wslot(i, r)] = h ? u[i][r].im : u[i][r].re;
          __syncthreads();
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const T x = lr[(sj + lds_skew<SK>(q * P)) * SI + b * SB];
            if (h) v[q].im = x;
            else v[q].re = x;
          }
        }
      } else {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int r = 0; r < R; ++r) lds[wslot(i, r)] = u[i][r];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < E; ++q) v[q] = lds[(sj + lds_skew<SK>(q * P)) * SI + b * SB];
      }
      fft_stages<T, L, E, INV, SI, SB, s + 1, SK, SPL>(v, lds, tw, b, j);
    }
  }
}

// Length-L transform of the lane's registers.  Contains __syncthreads() when
// the schedule has more than one stage: every lane of the block must call it.
template <typename T, int L, int E, bool INV, int SI, int SB, int SK = 0, bool SPL = false>
__device__ __forceinline__ void fft(cx<T> (&v)[E], cx<T>* lds, const cx<T>* tw, int b, int j) {
  fft_stages<T, L, E, INV, SI, SB, 0, SK, SPL>(v, lds, tw, b, j);
}

// ---------------------------------------------------------------------------
// Small reductions (wave64).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace ffcz
