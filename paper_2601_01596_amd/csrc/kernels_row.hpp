// Last-axis passes.  A block owns ROWS rows of the half-spectrum (H+1 complex
// entries each, H = n_last/2) and runs the real transforms through a complex
// transform of length H: the real row r is packed as z[m] = r[2m] + i r[2m+1].
//   C2R:  Z'[k] = (X[k] + X[H-k]*) + i W^-k (X[k] - X[H-k]*),  r = IDFT_H(Z') / n
//   R2C:  X[k] = (Z[k] + Z[H-k]*)/2 - i W^k (Z[k] - Z[H-k]*)/2,  X[H] = Re Z0 - Im Z0
// with W = exp(-2 pi i / n).  The imaginary parts of X[0] and X[H] are taken
// as zero, as a real inverse transform does.
//
// Three phases per block:
//   load     lanes walk the row tile in memory order (coalesced) into LDS;
//   compute  lane (row rl, j) with rows fastest: a wave touches up to 64 rows
//            at one index, and the odd LDS row pitch H+1 puts those rows on
//            distinct banks, so every Stockham exchange is conflict-free;
//            the spatial projection runs on registers between the two
//            transforms, so the spatial error never leaves the chip;
//   store    lanes walk the tile in memory order again, unpacking the R2C
//            output (or forming y = x + eps) on the way out.
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

// Move y one representable step toward x until |y - x| <= E holds in FP64.  The
// loop ends: every step moves y strictly toward x, and y = x satisfies the test for
// any E >= 0 (a NaN x or y fails the comparison and leaves at once).  With y the
// rounding of x + eps, |eps| <= E, it takes at most a step or two.
template <typename TIO>
__device__ __forceinline__ TIO closing_clamp(TIO y, TIO x, double E) {
  while (fabs((double)y - (double)x) > E) y = nextafter(y, x);
  return y;
}

// Long radix-16 rows need more than the 128 registers of four waves per SIMD.
__host__ __device__ constexpr int row_min_waves(int H, int E) { return (H >= 512 && E == 16) ? 3 : 4; }

template <typename T, typename TIO, int H, int ROWS, int MODE, int E>
__global__ void __launch_bounds__(ROWS*(H / E), row_min_waves(H, E))
row_kernel(RowArgs<T, TIO> a) {
  constexpr int P = H / E;
  constexpr int NT = ROWS * P;
  constexpr int LP = row_lds_pitch<T>(H, ROWS, E);               // LDS row pitch (entries)
  constexpr int SKW = row_lds_shift(H, ROWS, E, (int)sizeof(cx<T>));  // 0, or entry i at i + (i >> SKW)
  constexpr int NC = H + 1;            // spectrum entries per row
  using S = Sched<H, E>;
  constexpr int TW = S::twsize;
  constexpr int NW = (NT + 63) / 64;
  constexpr int SW = 2 * (H >= 32 ? H / 32 : 1);  // uint32 words per s-mask row (64-bit padded)
  using V2 = typename Vec2<TIO>::type;
  constexpr bool finalv = MODE == ROW_FINALV;  // FP64 fields only
  constexpr bool final_y = (MODE == ROW_FINAL || finalv || MODE == ROW_FINALP);  // forms and stores y
  constexpr bool decode = MODE == ROW_DECODE;  // y = x_hat + s + eps (s already in y)
  constexpr bool m_init = (MODE == ROW_INIT || MODE == ROW_INITE || MODE == ROW_INITP);
  constexpr bool m_loop = (MODE == ROW_LOOP || MODE == ROW_LOOPE || MODE == ROW_LOOPP);
  constexpr bool m_verify = (MODE == ROW_VERIFY || MODE == ROW_VERIFYP);
  constexpr bool sedit = (MODE == ROW_INITE || MODE == ROW_LOOPE);  // spatial edit bookkeeping
  // a spatial bound per point (E_n from st->pE, or the scalar when that is null)
  constexpr bool pwE = (MODE == ROW_INITP || MODE == ROW_LOOPP || MODE == ROW_FINALP || MODE == ROW_VERIFYP);
  constexpr bool spec_in = (m_loop || final_y || MODE == ROW_BLOOP || MODE == ROW_BFINAL || decode);
  constexpr bool spec_out = (m_init || m_loop || m_verify || MODE == ROW_BINIT ||
                             MODE == ROW_BLOOP || finalv);
  constexpr bool rec_s = (m_init || m_loop);
  constexpr bool use_s = (MODE == ROW_BINIT || MODE == ROW_BLOOP || MODE == ROW_BFINAL);
  // the final passes read the loop's spectrum in the field's precision (TIO), which is
  // the working precision except for an FP64 final of an FP32 field
  using SrcT = typename std::conditional<final_y, TIO, T>::type;
  const cx<SrcT>* src = reinterpret_cast<const cx<SrcT>*>(a.src);
  static_assert(!finalv || (sizeof(T) == 8 && sizeof(TIO) == 8), "the fused closing pass serves FP64 fields");

  __shared__ cx<T> lds[ROWS * LP];
  // rows of 1024 entries and more: the twiddle tables (about two rows' worth) are read
  // from global memory, where the caches hold them, so that more blocks fit a CU
  constexpr bool twg = H >= 1024;
  __shared__ cx<T> tws_l[twg ? 1 : TW + H];
  const cx<T>* tws = twg ? a.tw : tws_l;
  __shared__ unsigned long long red_u[NW];
  __shared__ double red_d[NW];
  __shared__ uint32_t sbits[(rec_s || use_s) ? ROWS * SW : 1];

  // block -> (instance, first row); blocks never straddle two instances
  const int64_t inst = (int64_t)blockIdx.x / a.bpi;
  const int64_t lrow0 = ((int64_t)blockIdx.x - inst * a.bpi) * ROWS;  // row within the instance
  const int64_t row0 = inst * a.rows_per_inst + lrow0;                 // row of the spectrum buffers
  DevState* st = a.st + inst;
  if constexpr (m_loop) {
    if (*(volatile int32_t*)&st->done) return;
  }
  // first entry of spectrum row R (rows are grouped in planes of 2^lg_rpp rows)
  auto rowaddr = [&](int64_t R) -> int64_t {
    return (R >> a.lg_rpp) * a.plane + (R & ((int64_t(1) << a.lg_rpp) - 1)) * a.pitch;
  };
  auto srowaddr = [&](int64_t R) -> int64_t {
    return (R >> a.lg_rpp) * a.splane + (R & ((int64_t(1) << a.lg_rpp) - 1)) * a.spitch;
  };
  const int t = threadIdx.x;
  const int rl = t % ROWS;  // compute mapping: rows fastest
  const int j = t / ROWS;
  const int nrow = (int)((a.rows_per_inst - lrow0) < ROWS ? (a.rows_per_inst - lrow0) : ROWS);
  cx<T>* lrow = lds + rl * LP;
  const int sj = lds_skew<SKW>(j);  // j < P, P a power of two: lds_skew<SKW>(j + qP) = sj + lds_skew<SKW>(qP)
  const cx<T>* rtw = tws + TW;

  if constexpr (!twg)
    for (int i = t; i < TW + H; i += NT) tws_l[i] = a.tw[i];

  int kround = 0;
  bool rec = false;
  if constexpr (rec_s) {
    if (m_loop) kround = *(volatile int32_t*)&st->round;
    rec = st->record_masks != 0;
    if (rec)
      for (int i = t; i < ROWS * SW; i += NT) sbits[i] = 0u;
  }
  if constexpr (use_s) {
    // the rows' mask words, coalesced
    for (int i = t; i < ROWS * SW; i += NT) {
      const int r = i / SW, w = i - r * SW;
      sbits[i] = (r < nrow && w < a.s_row_w32) ? a.smask[(row0 + r) * a.s_row_w32 + w] : 0u;
    }
  }
  if constexpr (rec_s || use_s) __syncthreads();  // mask words ready before any lane touches them
  // spatial edits of this instance (real point n of row R at R * 2H + n)
  T* const sed = sedit ? a.sedit + inst * a.rows_per_inst * (2 * H) : nullptr;

  unsigned long long cnt = 0;
  double mx = 0.0;
  // INIT: (x, x_hat); VERIFY: (x, y); BINIT: dL/dy in pxb; FINAL: x, writes y; BFINAL writes py
  const V2* x2 = reinterpret_cast<const V2*>(st->px);
  const V2* b2 = reinterpret_cast<const V2*>(m_verify ? (const void*)st->py : st->pxb);
  // pointwise spatial bounds, same layout and dtype as the fields
  const TIO* const pE = pwE ? reinterpret_cast<const TIO*>(st->pE) : nullptr;

  // ------------------------------------------------------------------ load
  // Unrolled in batches of BL so each lane keeps BL global loads in flight.
  constexpr int BL = 8;
  // FP32 spectra move two entries per 16-byte access: pair m of a row holds entries 2m, 2m+1
  // (the last pair of a row reaches into its padding, which is read but never written)
  constexpr bool pairs = sizeof(cx<T>) == 8 && H >= 2;
  constexpr bool pairs_in = sizeof(cx<SrcT>) == 8 && H >= 2;
  constexpr int NPR = (NC + 1) / 2;  // pairs per row
  // FP32 real fields move four reals (two packed entries) per 16-byte access
  constexpr bool io4 = sizeof(TIO) == 4 && H >= 2;
  constexpr int HQ = H / 2;  // 16-byte groups per real row
  if constexpr (spec_in && pairs_in) {
    constexpr int NLP = (ROWS * NPR + NT - 1) / NT;
    constexpr int BLP = NLP < 8 ? NLP : 8;  // loads per lane in flight
#pragma unroll
    for (int u0 = 0; u0 < NLP; u0 += BLP) {
      float4 tmp[BLP];
#pragma unroll
      for (int u = 0; u < BLP; ++u) {
        const int f = t + (u0 + u) * NT;
        const int r = f / NPR, m = f - r * NPR;
        tmp[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (u0 + u < NLP && f < ROWS * NPR && r < nrow)
          tmp[u] = *reinterpret_cast<const float4*>(src + srowaddr(row0 + r) + 2 * m);
      }
#pragma unroll
      for (int u = 0; u < BLP; ++u) {
        const int f = t + (u0 + u) * NT;
        if (u0 + u < NLP && f < ROWS * NPR) {
          const int r = f / NPR, m = f - r * NPR;
          lds[r * LP + lds_skew<SKW>(2 * m)] = cx<T>{(T)tmp[u].x, (T)tmp[u].y};
          if (2 * m + 1 < NC) lds[r * LP + lds_skew<SKW>(2 * m + 1)] = cx<T>{(T)tmp[u].z, (T)tmp[u].w};
        }
      }
    }
  } else if constexpr (spec_in) {
    constexpr int NL = (ROWS * NC + NT - 1) / NT;
#pragma unroll
    for (int b0 = 0; b0 < NL; b0 += BL) {
      cx<T> tmp[BL];
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int f = t + (b0 + u) * NT;
        const int r = f / NC, k = f - r * NC;
        tmp[u] = cx<T>{T(0), T(0)};
        if (b0 + u < NL && f < ROWS * NC && r < nrow) {
          const cx<SrcT> z = src[srowaddr(row0 + r) + k];
          tmp[u] = cx<T>{(T)z.re, (T)z.im};
        }
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int f = t + (b0 + u) * NT;
        if (b0 + u < NL && f < ROWS * NC) {
          const int r = f / NC, k = f - r * NC;
          lds[r * LP + lds_skew<SKW>(k)] = tmp[u];
        }
      }
    }
  } else {
    // real rows -> packed pairs; INIT also forms eps0 = x_hat - x in FP64 and clips it
    // spatial bound of INIT (the shrunk one) and VERIFY (the bound itself) when no array is given
    const double Ep = m_verify ? st->E : st->Ep;
    const double fe = st->fe;
    // packed entry m of row r from (x, second field) reals 2m, 2m+1; ep0, ep1: their spatial
    // bounds (INIT: shrunk; VERIFY: as given)
    auto pack = [&](int r, int m, double xa0, double xa1, double b0, double b1, double ep0,
                    double ep1) -> cx<T> {
      double e0 = 0.0, e1 = 0.0;
      if (r < nrow) {
        if constexpr (MODE == ROW_BINIT) {
          const uint32_t w = sbits[r * SW + (2 * m) / 32];
          const int sh = (2 * m) & 31;
          e0 = ((w >> sh) & 1u) ? b0 : 0.0;
          e1 = ((w >> (sh + 1)) & 1u) ? b1 : 0.0;
        } else {
          e0 = b0 - xa0;
          e1 = b1 - xa1;
          if constexpr (m_init) {
            const bool f0 = isfinite(e0), f1 = isfinite(e1);
            if (!f0 || !f1) {
              atomicAdd(&st->nonfinite, (unsigned long long)((!f0) + (!f1)));
              e0 = f0 ? e0 : 0.0;
              e1 = f1 ? e1 : 0.0;
            }
            const bool k0 = fabs(e0) <= ep0, k1 = fabs(e1) <= ep1;
            cnt += (!k0) + (!k1);
            const double c0 = clipv(e0, ep0), c1 = clipv(e1, ep1);
            if constexpr (sedit) {
              // the guard clip is the first ProjectOntoSCube displacement (every point written)
              typename Vec2<T>::type d;
              d.x = (T)(c0 - e0);
              d.y = (T)(c1 - e1);
              *reinterpret_cast<typename Vec2<T>::type*>(sed + (lrow0 + r) * (2 * H) + 2 * m) = d;
            }
            e0 = c0;
            e1 = c1;
            if (rec)
              atomicOr(&sbits[r * SW + (2 * m) / 32], ((uint32_t)k0 | ((uint32_t)k1 << 1)) << ((2 * m) & 31));
          } else if constexpr (MODE == ROW_VERIFYP) {
            // the largest ratio to the bound (0 / 0 counts as 0)
            const double r0 = e0 == 0.0 ? 0.0 : fabs(e0) / ep0, r1 = e1 == 0.0 ? 0.0 : fabs(e1) / ep1;
            mx = fmax(mx, fmax(r0, r1));
          } else {
            mx = fmax(mx, fmax(fabs(e0), fabs(e1)));
          }
        }
      }
      return cx<T>{(T)e0, (T)e1};  // rounded once to the working type
    };
    // the spatial bounds of reals 2m, 2m+1 from a loaded pair of E_n (INIT shrinks them)
    auto bnd = [&](double E0) -> double { return MODE == ROW_INITP ? E0 * fe : E0; };
    if constexpr (io4) {
      // FP32 fields: four reals (two packed entries) per 16-byte load, BQ loads of each field per
      // lane in flight (more spills: the FP64 difference, clip and mask work needs the registers)
      constexpr int NLQ = (ROWS * HQ + NT - 1) / NT;
      constexpr int BQ = NLQ < 4 ? NLQ : 4;
      const float4* x4 = reinterpret_cast<const float4*>(st->px);
      const float4* b4 = reinterpret_cast<const float4*>(m_verify ? (const void*)st->py : st->pxb);
      const float4* e4 = reinterpret_cast<const float4*>(pE);
#pragma unroll
      for (int q0 = 0; q0 < NLQ; q0 += BQ) {
        float4 xa[BQ], xbv[BQ];
        float4 ea[pwE ? BQ : 1];
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
          const int f = t + (q0 + u) * NT;
          const int r = f / HQ, q = f - r * HQ;
          const bool ok = q0 + u < NLQ && f < ROWS * HQ && r < nrow;
          const int64_t gi = (lrow0 + r) * HQ + q;
          xa[u] = make_float4(0.f, 0.f, 0.f, 0.f);
          xbv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
          if constexpr (MODE != ROW_BINIT) {
            if (ok) xa[u] = x4[gi];
          }
          if (ok) xbv[u] = b4[gi];
          if constexpr (pwE) {
            ea[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ok && e4) ea[u] = e4[gi];
          }
        }
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
          const int f = t + (q0 + u) * NT;
          if (!(q0 + u < NLQ && f < ROWS * HQ)) continue;
          const int r = f / HQ, q = f - r * HQ;
          double p0 = Ep, p1 = Ep, p2 = Ep, p3 = Ep;
          if constexpr (pwE) {
            if (e4) {
              p0 = bnd(ea[u].x);
              p1 = bnd(ea[u].y);
              p2 = bnd(ea[u].z);
              p3 = bnd(ea[u].w);
            }
          }
          lds[r * LP + lds_skew<SKW>(2 * q)] = pack(r, 2 * q, xa[u].x, xa[u].y, xbv[u].x, xbv[u].y, p0, p1);
          lds[r * LP + lds_skew<SKW>(2 * q + 1)] =
              pack(r, 2 * q + 1, xa[u].z, xa[u].w, xbv[u].z, xbv[u].w, p2, p3);
        }
      }
    } else {
      constexpr int NL = (ROWS * H + NT - 1) / NT;
#pragma unroll
      for (int b0 = 0; b0 < NL; b0 += BL) {
        V2 xa[BL], xbv[BL];
        V2 ea[pwE ? BL : 1];
        const V2* e2 = reinterpret_cast<const V2*>(pE);
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          const int r = f / H, m = f - r * H;
          const bool ok = b0 + u < NL && f < ROWS * H && r < nrow;
          const int64_t gi = (lrow0 + r) * H + m;
          if constexpr (MODE != ROW_BINIT) {
            if (ok) xa[u] = x2[gi];
          }
          if (ok) xbv[u] = b2[gi];
          if constexpr (pwE) {
            if (ok && e2) ea[u] = e2[gi];
          }
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          if (!(b0 + u < NL && f < ROWS * H)) continue;
          const int r = f / H, m = f - r * H;
          double p0 = Ep, p1 = Ep;
          if constexpr (pwE) {
            if (e2 && r < nrow) {
              p0 = bnd((double)ea[u].x);
              p1 = bnd((double)ea[u].y);
            }
          }
          lds[r * LP + lds_skew<SKW>(m)] =
              pack(r, m, (double)xa[u].x, (double)xa[u].y, (double)xbv[u].x, (double)xbv[u].y, p0, p1);
        }
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------ compute
  cx<T> v[E];
  if constexpr (spec_in) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      cx<T> A = lrow[sj + lds_skew<SKW>(q * P)];
      cx<T> B = lrow[lds_skew<SKW>(H - k)];
      if (k == 0) {
        A.im = T(0);
        B.im = T(0);
      }
      const cx<T> sm = A + conjg(B);
      const cx<T> df = cmulc(A - conjg(B), rtw[k]);  // W^-k (A - B*)
      v[q] = cx<T>{sm.re - df.im, sm.im + df.re};    // sm + i * df
    }
    fft<T, H, E, true, 1, LP, SKW>(v, lds, tws, rl, j);
    const T sc = (T)st->inv_n;
    if constexpr (final_y) {
      // the source holds only the last-axis R2C of eps, so the C2R scale is 1/n_last
      const T scz = T(1) / T(2 * H);
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = scal(v[q], scz);
    } else if constexpr (decode) {
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = scal(v[q], sc);
    } else if constexpr (MODE == ROW_BLOOP || MODE == ROW_BFINAL) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int k = j + q * P;
        const uint32_t w = sbits[rl * SW + (2 * k) / 32];
        const int sh = (2 * k) & 31;
        v[q].re = ((w >> sh) & 1u) ? v[q].re * sc : T(0);
        v[q].im = ((w >> (sh + 1)) & 1u) ? v[q].im * sc : T(0);
      }
    } else {  // ROW_LOOP: ProjectOntoSCube
      const T Ep = to_t<T>(st->Ep);
      const bool valid = rl < nrow;
      const V2* e2 = reinterpret_cast<const V2*>(pE);
      const double fe = st->fe;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int k = j + q * P;
        T e0 = v[q].re * sc, e1 = v[q].im * sc;
        T Ep0 = Ep, Ep1 = Ep;
        if constexpr (pwE) {
          // the bounds of reals 2k, 2k+1 of this row, shrunk (rounded toward zero in FP32)
          if (e2 && valid) {
            const V2 ev = e2[(lrow0 + rl) * H + k];
            Ep0 = to_t<T>((double)ev.x * fe);
            Ep1 = to_t<T>((double)ev.y * fe);
          }
        }
        const bool k0 = fabs(e0) <= Ep0, k1 = fabs(e1) <= Ep1;
        if (valid) cnt += (!k0) + (!k1);
        const T c0 = clipv(e0, Ep0), c1 = clipv(e1, Ep1);
        if constexpr (sedit) {
          // spat_edits += eps' - eps at the points the clip moved
          if (valid && !(k0 && k1)) {
            T* pe = sed + (lrow0 + rl) * (2 * H) + 2 * k;
            if (!k0) pe[0] += c0 - e0;
            if (!k1) pe[1] += c1 - e1;
          }
        }
        v[q] = cx<T>{c0, c1};
        if (rec && valid)
          atomicOr(&sbits[rl * SW + (2 * k) / 32], ((uint32_t)k0 | ((uint32_t)k1 << 1)) << ((2 * k) & 31));
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = lrow[sj + lds_skew<SKW>(q * P)];
  }
  if constexpr (spec_out && !finalv) fft<T, H, E, false, 1, LP, SKW>(v, lds, tws, rl, j);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) lrow[sj + lds_skew<SKW>(q * P)] = v[q];
  __syncthreads();

  // ------------------------------------------------------------------ store
  // entry k of the row's R2C output from the packed transform in LDS
  auto unpack = [&](const cx<T>* zr, int k) -> cx<T> {
    if (k == H) {
      const cx<T> z0 = zr[0];
      return cx<T>{z0.re - z0.im, T(0)};
    }
    const cx<T> Zk = zr[lds_skew<SKW>(k)];
    const cx<T> Zm = zr[lds_skew<SKW>((H - k) & (H - 1))];
    const cx<T> ev = scal(Zk + conjg(Zm), T(0.5));
    const cx<T> d = Zk - conjg(Zm);
    const cx<T> od = cx<T>{d.im * T(0.5), -d.re * T(0.5)};  // d / (2i)
    return ev + cmul(rtw[k], od);
  };
  if constexpr (!spec_out || finalv) {
    // ROW_FINAL / ROW_FINALV: y = x + eps formed in FP64, rounded once, clamped;  ROW_BFINAL:
    // store g.  ROW_FINALV puts d = y - x (FP64, from the stored y) back into the row's LDS
    // entries and keeps max |d|.
    V2* y2 = reinterpret_cast<V2*>(st->py);
    const double Eb = st->E;
    auto out_of = [&](TIO xv, T e, double Ebound) -> TIO {
      if constexpr (final_y) return closing_clamp<TIO>(round_io<TIO>((double)xv + (double)e), xv, Ebound);
      else return (TIO)e;
    };
    // decoder: x_hat from pxb, the expanded spatial edits already in y
    auto dec_of = [&](TIO xbv, TIO sv, T e) -> TIO { return round_io<TIO>((double)xbv + (double)sv + (double)e); };
    constexpr bool ld_x = final_y || decode;
    constexpr int NS = (ROWS * H + NT - 1) / NT;
    if constexpr (io4) {
      // FP32 fields: four reals per 16-byte access
      constexpr int NSQ = (ROWS * HQ + NT - 1) / NT;
      constexpr int BQ = NSQ < 8 ? NSQ : 8;
      const float4* x4 = reinterpret_cast<const float4*>(decode ? st->pxb : st->px);
      float4* y4 = reinterpret_cast<float4*>(st->py);
      const float4* e4 = reinterpret_cast<const float4*>(pE);
#pragma unroll
      for (int q0 = 0; q0 < NSQ; q0 += BQ) {
        float4 xa[BQ];
        float4 sa[decode ? BQ : 1];
        float4 ea[pwE ? BQ : 1];
        if constexpr (ld_x) {
#pragma unroll
          for (int u = 0; u < BQ; ++u) {
            const int f = t + (q0 + u) * NT;
            const int r = f / HQ, q = f - r * HQ;
            if (q0 + u < NSQ && f < ROWS * HQ && r < nrow) {
              xa[u] = x4[(lrow0 + r) * HQ + q];
              if constexpr (decode) sa[u] = y4[(lrow0 + r) * HQ + q];
              if constexpr (pwE) {
                const float Es = (float)Eb;  // unused when e4 is null
                ea[u] = e4 ? e4[(lrow0 + r) * HQ + q] : make_float4(Es, Es, Es, Es);
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
          const int f = t + (q0 + u) * NT;
          const int r = f / HQ, q = f - r * HQ;
          if (q0 + u < NSQ && f < ROWS * HQ && r < nrow) {
            const cx<T> e0 = lds[r * LP + lds_skew<SKW>(2 * q)], e1 = lds[r * LP + lds_skew<SKW>(2 * q + 1)];
            float4 o;
            if constexpr (pwE) {
              const bool ga = e4 != nullptr;
              o = make_float4(out_of(xa[u].x, e0.re, ga ? (double)ea[u].x : Eb),
                              out_of(xa[u].y, e0.im, ga ? (double)ea[u].y : Eb),
                              out_of(xa[u].z, e1.re, ga ? (double)ea[u].z : Eb),
                              out_of(xa[u].w, e1.im, ga ? (double)ea[u].w : Eb));
            } else if constexpr (final_y) {
              o = make_float4(out_of(xa[u].x, e0.re, Eb), out_of(xa[u].y, e0.im, Eb), out_of(xa[u].z, e1.re, Eb),
                              out_of(xa[u].w, e1.im, Eb));
            } else if constexpr (decode) {
              o = make_float4(dec_of(xa[u].x, sa[u].x, e0.re), dec_of(xa[u].y, sa[u].y, e0.im),
                              dec_of(xa[u].z, sa[u].z, e1.re), dec_of(xa[u].w, sa[u].w, e1.im));
            } else {
              o = make_float4((float)e0.re, (float)e0.im, (float)e1.re, (float)e1.im);
            }
            y4[(lrow0 + r) * HQ + q] = o;
          }
        }
      }
    } else {
    const V2* xd2 = reinterpret_cast<const V2*>(decode ? st->pxb : st->px);
    const V2* ed2 = reinterpret_cast<const V2*>(pE);
#pragma unroll
    for (int b0 = 0; b0 < NS; b0 += BL) {
      V2 xa[BL];
      V2 sa[decode ? BL : 1];
      double eb0[pwE ? BL : 1], eb1[pwE ? BL : 1];
      if constexpr (ld_x) {
#pragma unroll
        for (int u = 0; u < BL; ++u) {
          const int f = t + (b0 + u) * NT;
          const int r = f / H, m = f - r * H;
          if (b0 + u < NS && f < ROWS * H && r < nrow) {
            xa[u] = xd2[(lrow0 + r) * H + m];
            if constexpr (decode) sa[u] = y2[(lrow0 + r) * H + m];
            if constexpr (pwE) {
              eb0[u] = eb1[u] = Eb;
              if (ed2) {
                const V2 ev = ed2[(lrow0 + r) * H + m];
                eb0[u] = (double)ev.x;
                eb1[u] = (double)ev.y;
              }
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < BL; ++u) {
        const int f = t + (b0 + u) * NT;
        const int r = f / H, m = f - r * H;
        if (b0 + u < NS && f < ROWS * H && r < nrow) {
          const cx<T> e = lds[r * LP + lds_skew<SKW>(m)];
          V2 out;
          if constexpr (pwE) {
            out.x = out_of(xa[u].x, e.re, eb0[u]);
            out.y = out_of(xa[u].y, e.im, eb1[u]);
          } else if constexpr (final_y) {
            out.x = out_of(xa[u].x, e.re, Eb);
            out.y = out_of(xa[u].y, e.im, Eb);
          } else if constexpr (decode) {
            out.x = dec_of(xa[u].x, sa[u].x, e.re);
            out.y = dec_of(xa[u].y, sa[u].y, e.im);
          } else {
            out.x = (TIO)e.re;
            out.y = (TIO)e.im;
          }
          y2[(lrow0 + r) * H + m] = out;
          if constexpr (finalv) {
            const double d0 = (double)out.x - (double)xa[u].x, d1 = (double)out.y - (double)xa[u].y;
            mx = fmax(mx, fmax(fabs(d0), fabs(d1)));
            lds[r * LP + lds_skew<SKW>(m)] = cx<T>{(T)d0, (T)d1};
          }
        }
      }
    }
    }
  }
  if constexpr (finalv) {
    // FP64 R2C of d: each lane rewrites only LDS entries it read above, so the barrier
    // before the transform is the only one needed
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = lrow[sj + lds_skew<SKW>(q * P)];
    fft<T, H, E, false, 1, LP, SKW>(v, lds, tws, rl, j);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; ++q) lrow[sj + lds_skew<SKW>(q * P)] = v[q];
    __syncthreads();
  }
  if constexpr (spec_out && pairs) {
    constexpr int NSP = (ROWS * NPR + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < NSP; ++it) {
      const int f = t + it * NT;
      const int r = f / NPR, m = f - r * NPR;
      if (f < ROWS * NPR && r < nrow) {
        const cx<T>* zr = lds + r * LP;
        const cx<T> X0 = unpack(zr, 2 * m);
        // the last pair of a row holds entry H and the first padding entry of the row
        // (the pitch is a multiple of 16 above H + 1), stored as zero: every pair is one
        // 16-byte store (a branch with a lone 8-byte store gets split into 4 + 12 bytes)
        cx<T> X1{T(0), T(0)};
        if (2 * m + 1 < NC) X1 = unpack(zr, 2 * m + 1);
        *reinterpret_cast<float4*>(a.dst + rowaddr(row0 + r) + 2 * m) =
            make_float4((float)X0.re, (float)X0.im, (float)X1.re, (float)X1.im);
      }
    }
  } else if constexpr (spec_out) {
    constexpr int NS = (ROWS * NC + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < NS; ++it) {
      const int f = t + it * NT;
      const int r = f / NC, k = f - r * NC;
      if (f < ROWS * NC && r < nrow) a.dst[rowaddr(row0 + r) + k] = unpack(lds + r * LP, k);
    }
  }

  // ------------------------------------------------------------------ partials and masks
  if constexpr (m_init || m_loop || m_verify || finalv) {
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
      if constexpr (m_verify || finalv) a.part[blockIdx.x] = (unsigned long long)__double_as_longlong(m);
      else a.part[blockIdx.x] = s;
    }
    if constexpr (rec_s) {
      if (rec) {
        uint32_t* plane = a.smask + (int64_t)kround * a.s_plane;
        for (int i = t; i < ROWS * SW; i += NT) {
          const int r = i / SW;
          const int w = i - r * SW;
          if (r < nrow && w < a.s_row_w32) plane[(row0 + r) * a.s_row_w32 + w] = sbits[i];
        }
      }
    }
  }
}

}  // namespace ffcz

namespace ffcz {

// The value z of lane (P - j) mod P of the lane's group (j = lane mod P), through the
// LDS crossbar (ds_bpermute: no LDS storage, no barrier); baddr = 4 x that lane's index
// in the wave.  Lane 0 of a group reads its own z.
__device__ __forceinline__ cx<float> lane_read(cx<float> z, int baddr) {
  return cx<float>{__int_as_float(__builtin_amdgcn_ds_bpermute(baddr, __float_as_int(z.re))),
                   __int_as_float(__builtin_amdgcn_ds_bpermute(baddr, __float_as_int(z.im)))};
}

// Row pitch (entries) of the direct passes: H entries skewed as i + (i >> log2 P),
// rounded up to = P mod 32 8-byte slots, so the 64 / P rows of a wave fill every
// slot exactly twice in the transform's exchange (write: entry P r + ..., read:
// entry j + P q).
__host__ __device__ constexpr int direct_lds_pitch(int H) {
  const int P = H / 16;
  const int need = (H - 1) + ((H - 1) >> ilog2c(P)) + 1;
  int lp = need;
  while (lp % 32 != P % 32) ++lp;
  return lp;
}

// Last-axis passes for FP32 rows of H = 128 or 256 entries with lanes
// index-fastest: the P = H / 16 lanes of a row are one group of a wave, lane j
// keeps entries j + P q (q < 16).  Spectrum entries (and the real pairs r[2m],
// r[2m+1] of the fields) move straight between HBM and registers (P lanes cover 8 P
// contiguous bytes of a row per access), the C2R and R2C partners k <-> H - k come
// from lane (P - j) mod P through ds_bpermute, and LDS carries only the transform's own
// exchange, with entry i at i + (i >> log2 P) and rows direct_lds_pitch(H) apart
// (every 8-byte slot taken exactly twice per wave access).  row_kernel stages the
// whole tile through LDS on the way in and out; the loop pass moves about 40 % less
// LDS data this way.  Modes: ROW_INIT, ROW_LOOP, ROW_FINAL and the adjoint's
// ROW_BINIT, ROW_BLOOP, ROW_BFINAL, with row_kernel's formulas; the compiler fuses
// multiply-adds differently in the two kernels, so results can differ in the last
// bit (a plan that rounds differently, like radix 8).
template <int MODE, int H, int ROWS>
__global__ void __launch_bounds__(ROWS * (H / 16), 4) row_direct_kernel(RowArgs<float, float> a) {
  using T = float;
  constexpr int E = 16, P = H / E;
  constexpr int NT = ROWS * P;
  constexpr int SKW = ilog2c(P);
  constexpr int LP = direct_lds_pitch(H);
  using S = Sched<H, E>;
  constexpr int TW = S::twsize;
  constexpr int NW = (NT + 63) / 64;
  constexpr int SW = 2 * (H / 32);
  constexpr bool rec_s = (MODE == ROW_INIT || MODE == ROW_LOOP);
  constexpr bool use_s = (MODE == ROW_BINIT || MODE == ROW_BLOOP || MODE == ROW_BFINAL);
  constexpr bool spec_in = (MODE == ROW_LOOP || MODE == ROW_FINAL || MODE == ROW_BLOOP || MODE == ROW_BFINAL);
  constexpr bool spec_out = (MODE == ROW_INIT || MODE == ROW_LOOP || MODE == ROW_BINIT || MODE == ROW_BLOOP);
  static_assert(H == 128 || H == 256, "rows of 128 or 256 entries");
  static_assert(MODE != ROW_VERIFY, "the verification runs in FP64");
  static_assert(S::nst == 2, "one exchange per transform");

  // Rows of 128 entries exchange the real parts, then the imaginary parts, through one real
  // per entry: half the LDS, so more blocks share a CU (the full-width exchange held these
  // blocks to 12 waves per CU)
  constexpr bool SPX = (H == 128);
  __shared__ cx<T> lds[SPX ? (ROWS * LP + 1) / 2 : ROWS * LP];
  __shared__ cx<T> tws[TW + H];
  __shared__ unsigned long long red_u[NW];
  __shared__ uint32_t sbits[(rec_s || use_s) ? ROWS * SW : 1];

  const int64_t inst = (int64_t)blockIdx.x / a.bpi;
  const int64_t lrow0 = ((int64_t)blockIdx.x - inst * a.bpi) * ROWS;
  const int64_t row0 = inst * a.rows_per_inst + lrow0;
  DevState* st = a.st + inst;
  if constexpr (MODE == ROW_LOOP) {
    if (*(volatile int32_t*)&st->done) return;
  }
  auto rowaddr = [&](int64_t R) -> int64_t {
    return (R >> a.lg_rpp) * a.plane + (R & ((int64_t(1) << a.lg_rpp) - 1)) * a.pitch;
  };
  auto srowaddr = [&](int64_t R) -> int64_t {
    return (R >> a.lg_rpp) * a.splane + (R & ((int64_t(1) << a.lg_rpp) - 1)) * a.spitch;
  };
  const int t = threadIdx.x;
  const int j = t & (P - 1);
  const int rl = t / P;
  const int nrow = (int)((a.rows_per_inst - lrow0) < ROWS ? (a.rows_per_inst - lrow0) : ROWS);
  // Lanes past the block's last row (only in an instance's last block) repeat that row:
  // same loads, same arithmetic, so their stores write the same bytes to the same
  // addresses, and loads and stores need no per-lane guard; they count nothing and
  // record no mask bits.  They keep their own LDS row for the exchange.
  const bool valid = rl < nrow;
  const int rr = valid ? rl : nrow - 1;
  const cx<T>* rtw = tws + TW;
  // ds_bpermute address of lane (P - j) mod P of this lane's group, the C2R / R2C partner
  const int paddr = 4 * (((t & 63) & ~(P - 1)) | ((P - j) & (P - 1)));
  const int64_t g0 = (lrow0 + rr) * H;  // first real pair of the row in the fields
  // s-mask bits 2m, 2m+1 of this row (real pair m)
  auto sbit = [&](int m, int b) -> bool { return (sbits[rr * SW + (2 * m) / 32] >> (((2 * m) & 31) + b)) & 1u; };

  for (int i = t; i < TW + H; i += NT) tws[i] = a.tw[i];
  int kround = 0;
  bool rec = false;
  if constexpr (rec_s) {
    if (MODE == ROW_LOOP) kround = *(volatile int32_t*)&st->round;
    rec = st->record_masks != 0;
    if (rec)
      for (int i = t; i < ROWS * SW; i += NT) sbits[i] = 0u;
  }
  if constexpr (use_s) {
    // the rows' mask words, coalesced
    for (int i = t; i < ROWS * SW; i += NT) {
      const int r = i / SW, w = i - r * SW;
      sbits[i] = (r < nrow && w < a.s_row_w32) ? a.smask[(row0 + r) * a.s_row_w32 + w] : 0u;
    }
  }
  uint32_t cnt = 0;   // per lane, at most 2 E
  uint32_t wcnt = 0;  // per wave (the same in every lane)
  cx<T> v[E];
  const int64_t rbase = rowaddr(row0 + rr);
  // scale of the R2C's output: 1/2, times 1/N in the loop passes (N a product of
  // power-of-two extents, so moving 1/N past the clip and the transform changes no bit
  // beyond the transform's own rounding)
  T hsc = T(0.5);

  if constexpr (MODE == ROW_INIT) {
    // eps0 = x_hat - x in FP64 for the real pairs m = j + P q, guard clip (+ s-mask)
    const float2* x2 = reinterpret_cast<const float2*>(st->px);
    const float2* b2 = reinterpret_cast<const float2*>(st->pxb);
    const double Ep = st->Ep;
    __syncthreads();  // cleared mask words visible
    // two batches of 8 pairs per field (all 16 of both fields do not fit the registers
    // next to the FP64 arithmetic)
    constexpr int BQ = 8;
    float2 xa[BQ], xb[BQ];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (q % BQ == 0) {
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
          xa[u] = x2[g0 + j + (q + u) * P];
          xb[u] = b2[g0 + j + (q + u) * P];
        }
      }
      const int m = j + q * P;
      const int u = q % BQ;
      double e0 = (double)xb[u].x - (double)xa[u].x, e1 = (double)xb[u].y - (double)xa[u].y;
      const bool f0 = isfinite(e0), f1 = isfinite(e1);
      if (!f0 || !f1) {
        if (valid) atomicAdd(&st->nonfinite, (unsigned long long)((!f0) + (!f1)));
        e0 = f0 ? e0 : 0.0;
        e1 = f1 ? e1 : 0.0;
      }
      const bool k0 = fabs(e0) <= Ep, k1 = fabs(e1) <= Ep;
      cnt += (uint32_t)(!k0) + (uint32_t)(!k1);
      e0 = clipv(e0, Ep);
      e1 = clipv(e1, Ep);
      if (rec && valid)
        atomicOr(&sbits[rl * SW + (2 * m) / 32], ((uint32_t)k0 | ((uint32_t)k1 << 1)) << ((2 * m) & 31));
      v[q] = cx<T>{(T)e0, (T)e1};
    }
  } else if constexpr (MODE == ROW_BINIT) {
    // g * s-mask for the real pairs m = j + P q (dL/dy arrives in pxb)
    const float2* g2 = reinterpret_cast<const float2*>(st->pxb);
    float2 gv[E];
#pragma unroll
    for (int q = 0; q < E; ++q) gv[q] = g2[g0 + j + q * P];
    __syncthreads();  // mask words visible
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int m = j + q * P;
      v[q] = cx<T>{sbit(m, 0) ? gv[q].x : T(0), sbit(m, 1) ? gv[q].y : T(0)};
    }
  } else {
    static_assert(spec_in, "");
    // spectrum entries j + P q of the row, and the Nyquist entry for lane 0
    cx<T> x[E];
    cx<T> nyq{T(0), T(0)};
#pragma unroll
    for (int q = 0; q < E; ++q) x[q] = a.src[rbase + j + q * P];
    if (j == 0) nyq = a.src[rbase + H];
    __syncthreads();  // twiddles (and mask words) visible
    // C2R: Z'[k] = (X[k] + X[H-k]*) + i W^-k (X[k] - X[H-k]*), with d = X[k] - X[H-k]*:
    // Re Z' = Re s - Im d Re W + Re d Im W, Im Z' = Im s + Re d Re W + Im d Im W
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      cx<T> A = x[q];
      // X[H - k] is entry E-1-q of lane P-j; for j = 0 it is this lane's entry
      // (E-q) mod E (the Nyquist entry for q = 0), which lane 0 sends to itself
      const cx<T> own = (q == 0) ? nyq : x[(E - q) & (E - 1)];
      cx<T> B = lane_read((j == 0) ? own : x[E - 1 - q], paddr);
      if (k == 0) {
        A.im = T(0);
        B.im = T(0);
      }
      const cx<T> w = rtw[k];
      const T sre = A.re + B.re, sim = A.im - B.im;
      const T dre = A.re - B.re, dim = A.im + B.im;
      v[q] = cx<T>{__builtin_fmaf(dre, w.im, __builtin_fmaf(-dim, w.re, sre)),
                   __builtin_fmaf(dim, w.im, __builtin_fmaf(dre, w.re, sim))};
    }
    fft<T, H, E, true, 1, LP, SKW, SPX>(v, lds, tws, rl, j);
    if constexpr (MODE == ROW_LOOP) {
      // ProjectOntoSCube (+ s-mask) on N eps: the bound scaled by N, and 1/N applied by
      // the R2C below
      const T sc = (T)st->inv_n;
      const T Ep = to_t<T>(st->Ep) / sc;
      hsc = T(0.5) * sc;
      if (rec) {
        if (valid) {
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const int k = j + q * P;
            const bool k0 = fabs(v[q].re) <= Ep, k1 = fabs(v[q].im) <= Ep;
            atomicOr(&sbits[rl * SW + (2 * k) / 32], ((uint32_t)k0 | ((uint32_t)k1 << 1)) << ((2 * k) & 31));
          }
        }
      }
      // the count per wave: a ballot per value and a scalar popcount (the lanes of rows
      // past the block's end masked off)
      const unsigned long long vm = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        wcnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(!(fabs(v[q].re) <= Ep)) & vm);
        wcnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(!(fabs(v[q].im) <= Ep)) & vm);
        v[q] = cx<T>{clipv(v[q].re, Ep), clipv(v[q].im, Ep)};
      }
    } else if constexpr (MODE == ROW_FINAL) {
      // the source holds only the last-axis R2C of eps, so the C2R scale is 1/n_last
      const T scz = T(1) / T(2 * H);
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = scal(v[q], scz);
    } else {
      // adjoint: g * s-mask and 1/N (in the loop pass, 1/N is applied by the R2C below)
      const T sc = (T)st->inv_n;
      if constexpr (MODE == ROW_BLOOP) hsc = T(0.5) * sc;
      const T sv = MODE == ROW_BLOOP ? T(1) : sc;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int k = j + q * P;
        v[q].re = sbit(k, 0) ? v[q].re * sv : T(0);
        v[q].im = sbit(k, 1) ? v[q].im * sv : T(0);
      }
    }
  }

  if constexpr (MODE == ROW_FINAL || MODE == ROW_BFINAL) {
    // FINAL: y = x + eps formed in FP64, rounded once, clamped (closing clamp);
    // BFINAL: the gradient pairs
    float2* y2 = reinterpret_cast<float2*>(st->py);
    if constexpr (MODE == ROW_FINAL) {
      const float2* x2 = reinterpret_cast<const float2*>(st->px);
      const double Eb = st->E;
      // the loads of x in two batches of 8, each issued before its clamps (the clamp's
      // loop between loads would otherwise serialise them; 16 at once spill)
      constexpr int BQ = 8;
      float2 xv[BQ];
#pragma unroll
      for (int q0 = 0; q0 < E; q0 += BQ) {
#pragma unroll
        for (int u = 0; u < BQ; ++u) xv[u] = x2[g0 + j + (q0 + u) * P];
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
          const int q = q0 + u;
          if (valid)
            y2[g0 + j + q * P] =
                make_float2(closing_clamp<float>(round_io<float>((double)xv[u].x + (double)v[q].re), xv[u].x, Eb),
                            closing_clamp<float>(round_io<float>((double)xv[u].y + (double)v[q].im), xv[u].y, Eb));
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) y2[g0 + j + q * P] = make_float2(v[q].re, v[q].im);
    }
  } else {
    static_assert(spec_out, "");
    fft<T, H, E, false, 1, LP, SKW, SPX>(v, lds, tws, rl, j);
    // R2C: X[k] = (Z[k] + Z[H-k]*)/2 - i W^k (Z[k] - Z[H-k]*)/2, X[H] = Re Z0 - Im Z0,
    // times the pass's scale c (hsc = c/2); with s = Z[k] + Z[H-k]*, d = Z[k] - Z[H-k]*:
    // Re X = c/2 (Re s + Re W Im d + Im W Re d), Im X = c/2 (Im s - Re W Re d + Im W Im d)
    cx<T>* dst = a.dst + rbase;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = j + q * P;
      const cx<T> Zk = v[q];
      const cx<T> own = v[(E - q) & (E - 1)];  // lane 0: Z[H - P q], Z[0] for q = 0
      const cx<T> Zm = lane_read((j == 0) ? own : v[E - 1 - q], paddr);
      const cx<T> w = rtw[k];
      const T sre = Zk.re + Zm.re, sim = Zk.im - Zm.im;
      const T dre = Zk.re - Zm.re, dim = Zk.im + Zm.im;
      dst[k] = cx<T>{hsc * __builtin_fmaf(w.im, dre, __builtin_fmaf(w.re, dim, sre)),
                     hsc * __builtin_fmaf(w.im, dim, __builtin_fmaf(-w.re, dre, sim))};
    }
    // entry H and the row's first padding entry (zero) as one 16-byte store
    if (j == 0) *reinterpret_cast<float4*>(dst + H) = make_float4((hsc + hsc) * (v[0].re - v[0].im), 0.f, 0.f, 0.f);
  }

  if constexpr (rec_s) {
    // one partial per block (guard-clip or s-clip count), reduced by the control kernel
    unsigned long long wc = wcnt;
    if constexpr (MODE == ROW_INIT) wc = wave_sum_u64(valid ? (unsigned long long)cnt : 0ull);
    if ((t & 63) == 0) red_u[t >> 6] = wc;
    __syncthreads();
    if (t == 0) {
      unsigned long long s2 = 0;
      for (int w = 0; w < NW; ++w) s2 += red_u[w];
      a.part[blockIdx.x] = s2;
    }
    if (rec) {
      uint32_t* plane = a.smask + (int64_t)kround * a.s_plane;
      for (int i = t; i < ROWS * SW; i += NT) {
        const int r = i / SW;
        const int w = i - r * SW;
        if (r < nrow && w < a.s_row_w32) plane[(row0 + r) * a.s_row_w32 + w] = sbits[i];
      }
    }
  }
}

}  // namespace ffcz
