// Strided-axis passes.  A block owns C contiguous columns of one outer index
// and the whole transformed axis (length L): element (c, i) is read from
// src[outer*so + col0 + c + i*s], so every row of the tile is one 64-128 B
// contiguous segment.  Lane (j, c) keeps elements i = j + q*P of column c.
#pragma once
#include "common.hpp"

namespace ffcz {

template <typename T, int L, int C, int MODE>
__global__ void __launch_bounds__(C*(L / pick_E(L)))
col_kernel(ColArgs<T> a) {
  constexpr int E = pick_E(L);
  constexpr int P = L / E;
  constexpr int NT = C * P;
  using S = Sched<L, E>;
  constexpr int TW = S::twsize;
  constexpr int NW = (NT + 63) / 64;
  // the FP64 verification pass stores nothing, so registers allow four blocks per CU;
  // its exchange goes through LDS one real part at a time to let them fit
  constexpr bool SPL = ((MODE == COL_VERIFY || MODE == COL_VERIFYP) && sizeof(T) == 8);
  __shared__ cx<T> lds[S::nst > 1 ? (SPL ? L * C / 2 : L * C) : 1];
  __shared__ cx<T> tws[TW > 0 ? TW : 1];
  __shared__ unsigned long long red_u[NW];
  __shared__ double red_d[NW];

  const int64_t bid = xcd_tile(blockIdx.x, gridDim.x, a.xcd_k);
  const int64_t o = bid / a.ncb;
  DevState* st = a.st + o / a.outer_per_inst;
  constexpr bool uses_done =
      (MODE == COL_FWD || MODE == COL_INV || MODE == COL_XPASS || MODE == COL_XEDIT || MODE == COL_XPASSP);
  (void)red_d;
  if (uses_done) {
    if (*(volatile int32_t*)&st->done) return;
  }
  const int t = threadIdx.x;
  const int c = t % C;
  const int j = t / C;
  const int cb = (int)(bid - o * a.ncb);
  const int col = cb * C + c;
  const bool valid = col < a.ncols;
  // A padding column of the row (past the last column, inside the padded row) is stored as
  // zero: every line a pass writes is then whole (a store of part of a line cost about as
  // much as the whole line, 12 % of a strided pass for the row-end line).  Padding never
  // carries data.
  const bool padcol = !valid && col < a.ncols_pad;
  const int64_t base = o * a.so + col;
  // The x-direction passes (VALU-bound: two transforms per pass) address an entry as a
  // block-uniform part (outer index and row q P) plus a lane part (column and row j, in
  // bytes), one 64-bit add per access instead of a 64-bit multiply-add, and lanes past the
  // last column read that column (no per-lane guard on loads; they store nothing and count
  // nothing).  The other passes, with VALU to spare,
  // keep 64-bit indices and guarded loads, which timed faster for them.
  constexpr bool lean = (MODE == COL_XPASS || MODE == COL_XEDIT || MODE == COL_XUNDO ||
                         MODE == COL_XBACK || MODE == COL_XPASSP);
  const int col_in = valid ? col : a.ncols - 1;
  const int64_t lob = ((int64_t)col_in + (int64_t)j * a.s) * (int64_t)sizeof(cx<T>);
  const int64_t ob = o * a.so;
  auto src_at = [&](int q) -> const cx<T>* {
    return reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(a.src + ob + (int64_t)(q * P) * a.s) + lob);
  };
  const int64_t pad_b = (int64_t)(col - col_in) * (int64_t)sizeof(cx<T>);  // the lane's own column, for its stores
  auto dst_at = [&](int q) -> cx<T>* {
    return reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(a.dst + ob + (int64_t)(q * P) * a.s) + lob + pad_b);
  };

  for (int i = t; i < TW; i += NT) tws[i] = a.tw[i];

  cx<T> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    if constexpr (lean) v[q] = *src_at(q);
    else v[q] = valid ? a.src[base + (int64_t)(j + q * P) * a.s] : cx<T>{T(0), T(0)};
  }

  if constexpr (MODE == COL_FWD || MODE == COL_FWD_NS) {
    fft<T, L, E, false, C, 1>(v, lds, tws, c, j);
  } else if constexpr (MODE == COL_INV || MODE == COL_INV_NS) {
    fft<T, L, E, true, C, 1>(v, lds, tws, c, j);
  } else if constexpr (MODE == COL_XPASSP) {
    // pointwise bounds: entry k is checked against D_k fc and projected onto D_k fp, on Re and
    // Im separately (box) or on the modulus (disk, radial projection); no masks
    const T* bp = reinterpret_cast<const T*>(a.bnd);
    const int64_t bbase = o * a.bnd_so + col;
    const double fc = st->fc, fp = st->fp;
    const bool disk = st->disk != 0;
    fft<T, L, E, false, C, 1>(v, lds, tws, c, j);
    unsigned long long cnt = 0;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      cx<T> z = v[q];
      const int64_t bi = valid ? 2 * (bbase + (int64_t)(j + q * P) * a.bnd_s) : 0;
      const T br = valid ? bp[bi] : T(0), bim = valid ? bp[bi + 1] : T(0);
      if (disk) {
        const T m = hypot(z.re, z.im);
        const T dc = to_t<T>((double)br * fc), dp = to_t<T>((double)br * fp);
        cnt += (valid && m > dc) ? 1 : 0;
        if (m > dp) {
          const T sc = dp / m;
          z.re *= sc;
          z.im *= sc;
        }
      } else {
        const T dcr = to_t<T>((double)br * fc), dpr = to_t<T>((double)br * fp);
        const T dci = to_t<T>((double)bim * fc), dpi = to_t<T>((double)bim * fp);
        cnt += (valid && (fabs(z.re) > dcr || fabs(z.im) > dci)) ? 1 : 0;
        z.re = clipv(z.re, dpr);
        z.im = clipv(z.im, dpi);
      }
      v[q] = z;
    }
    fft<T, L, E, true, C, 1>(v, lds, tws, c, j);
    cnt = wave_sum_u64(cnt);
    if ((t & 63) == 0) red_u[t >> 6] = cnt;
    __syncthreads();
    if (t == 0) {
      unsigned long long s = 0;
      for (int w = 0; w < NW; ++w) s += red_u[w];
      a.part[bid] = s;
    }
  } else if constexpr (MODE == COL_XPASS || MODE == COL_XEDIT || MODE == COL_XUNDO) {
    // COL_XEDIT adds every clip displacement to the frequency edits (Alg. 1 edit bookkeeping);
    // COL_XUNDO repeats the forward transform and the clip of the check that ended the loop
    // (same inputs, same arithmetic, so the same displacements) and takes them back out: that
    // check's clip never reaches the iterate
    constexpr bool edit = MODE == COL_XEDIT, undo = MODE == COL_XUNDO;
    const int k = *(volatile int32_t*)&st->round;
    const T D = to_t<T>(st->Dc);
    const T Dp = to_t<T>(st->Dp);
    const bool rec = !undo && st->record_masks && (k < st->max_iter);
    fft<T, L, E, false, C, 1>(v, lds, tws, c, j);
    uint32_t wcnt = 0;  // violations of the wave (a ballot per entry, a scalar popcount)
    const int lane = t & 63;
    uint8_t* mre = a.fmask + (int64_t)k * 2 * a.f_plane;
    uint8_t* mim = mre + a.f_plane;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      cx<T> z = v[q];
      const bool bad = valid && (fabs(z.re) > D || fabs(z.im) > D);
      wcnt += (uint32_t)__popcll(__ballot(bad));
      const bool kre = fabs(z.re) <= Dp;
      const bool kim = fabs(z.im) <= Dp;
      z.re = clipv(z.re, Dp);
      z.im = clipv(z.im, Dp);
      if constexpr (edit || undo) {
        // displacement delta' - delta, touched only where the clip moved a part
        const T dre = z.re - v[q].re, dim = z.im - v[q].im;
        if (valid && (dre != T(0) || dim != T(0))) {
          cx<T>* f = a.fedit + base + (int64_t)(j + q * P) * a.s;
          cx<T> acc = *f;
          if constexpr (edit) {
            acc.re += dre;
            acc.im += dim;
          } else {
            acc.re -= dre;
            acc.im -= dim;
          }
          *f = acc;
        }
      }
      v[q] = z;
      if (rec) {
        const unsigned long long bre = __ballot(valid && kre);
        const unsigned long long bim = __ballot(valid && kim);
        if (c == 0 && cb * C < a.ncols) {  // a padding tile holds no column
          const int64_t row = (int64_t)(j + q * P) * a.mrow_i + o * a.mrow_o;
          const int64_t off = row * a.f_row_bytes + (cb * C) / 8;
          if constexpr (C == 16) {
            *(uint16_t*)(mre + off) = (uint16_t)((bre >> lane) & 0xFFFFull);
            *(uint16_t*)(mim + off) = (uint16_t)((bim >> lane) & 0xFFFFull);
          } else if constexpr (C == 8) {
            mre[off] = (uint8_t)((bre >> lane) & 0xFFull);
            mim[off] = (uint8_t)((bim >> lane) & 0xFFull);
          }
        }
      }
    }
    if constexpr (undo) return;
    fft<T, L, E, true, C, 1>(v, lds, tws, c, j);
    // violations of this check: one partial per block, summed by the control kernel
    if ((t & 63) == 0) red_u[t >> 6] = wcnt;
    __syncthreads();
    if (t == 0) {
      unsigned long long s = 0;
      for (int w = 0; w < NW; ++w) s += red_u[w];
      a.part[bid] = s;
    }
  } else if constexpr (MODE == COL_XBACK) {
    // The tile's f-mask bits of row j + q P are one C-bit word per plane (bit c: column
    // cb C + c).  Lane c of the C lanes of row group j loads the (Re, Im) words of the rows
    // with q = c (mod C), and the group reads them from that lane through the LDS crossbar
    // (ds_bpermute), in place of a byte load per entry and plane.
    // (Tiles of fewer than 8 columns read a byte per entry.)
    constexpr int WB = C >= 8 ? C / 8 : 1;  // mask bytes per tile row
    static_assert(C < 8 || WB == 1 || WB == 2, "tiles of 8 or 16 columns");
    constexpr int NWD = C >= 8 ? (E + C - 1) / C : 1;
    uint32_t wd[NWD];
    const bool tile_ok = cb * C < a.ncols;  // a padding tile has no mask bytes
    if constexpr (C >= 8) {
#pragma unroll
      for (int m = 0; m < NWD; ++m) {
        const int q = c + m * C;
        wd[m] = 0u;
        if (tile_ok && q < E) {
          const int64_t off = ((int64_t)(j + q * P) * a.mrow_i + o * a.mrow_o) * a.f_row_bytes + (cb * C) / 8;
          if constexpr (WB == 2)
            wd[m] = (uint32_t)*reinterpret_cast<const uint16_t*>(a.fmask + off) |
                    ((uint32_t)*reinterpret_cast<const uint16_t*>(a.fmask + a.f_plane + off) << 16);
          else
            wd[m] = (uint32_t)a.fmask[off] | ((uint32_t)a.fmask[a.f_plane + off] << 8);
        }
      }
    }
    fft<T, L, E, false, C, 1>(v, lds, tws, c, j);
    if constexpr (C >= 8) {
      const int gbase = (t & 63) & ~(C - 1);  // first lane of this row group in the wave
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const uint32_t w = (uint32_t)__builtin_amdgcn_ds_bpermute(4 * (gbase | (q % C)), (int)wd[q / C]);
        v[q].re = ((w >> c) & 1u) ? v[q].re : T(0);
        v[q].im = ((w >> (c + 8 * WB)) & 1u) ? v[q].im : T(0);
      }
    } else {
      const uint8_t* mre = a.fmask;
      const uint8_t* mim = a.fmask + a.f_plane;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int64_t off = ((int64_t)(j + q * P) * a.mrow_i + o * a.mrow_o) * a.f_row_bytes + col / 8;
        const int bit = col & 7;
        const int kr = valid ? (mre[off] >> bit) & 1 : 0;
        const int ki = valid ? (mim[off] >> bit) & 1 : 0;
        v[q].re = kr ? v[q].re : T(0);
        v[q].im = ki ? v[q].im : T(0);
      }
    }
    fft<T, L, E, true, C, 1>(v, lds, tws, c, j);
  } else if constexpr (MODE == COL_VERIFY || MODE == COL_VERIFYP) {
    fft<T, L, E, false, C, 1, 0, SPL>(v, lds, tws, c, j);
    const double D = st->Delta;
    unsigned long long cnt = 0;
    double mx = 0.0;
    if constexpr (MODE == COL_VERIFY) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        if (valid) {
          const double m = fmax(fabs((double)v[q].re), fabs((double)v[q].im));
          mx = fmax(mx, m);
          cnt += (m > D) ? 1 : 0;
        }
      }
    } else {
      // the largest ratio to the bound (0 / 0 counts as 0) and the entries above their bound
      const bool disk = st->disk != 0;
      const int64_t bbase = o * a.bnd_so + col;
      auto ratio = [](double x, double b) -> double { return x == 0.0 ? 0.0 : x / b; };
#pragma unroll
      for (int q = 0; q < E; ++q) {
        if (valid) {
          const int64_t bi = 2 * (bbase + (int64_t)(j + q * P) * a.bnd_s);
          const double br = a.bnd_dbl ? ((const double*)a.bnd)[bi] : (double)((const float*)a.bnd)[bi];
          const double bim = a.bnd_dbl ? ((const double*)a.bnd)[bi + 1] : (double)((const float*)a.bnd)[bi + 1];
          const double re = fabs((double)v[q].re), im = fabs((double)v[q].im);
          if (disk) {
            const double m = hypot(re, im);
            mx = fmax(mx, ratio(m, br));
            cnt += (m > br) ? 1 : 0;
          } else {
            mx = fmax(mx, fmax(ratio(re, br), ratio(im, bim)));
            cnt += (re > br || im > bim) ? 1 : 0;
          }
        }
      }
    }
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
      a.part[bid] = s;
      a.part[a.part_stride + bid] = (unsigned long long)__double_as_longlong(m);
    }
    return;
  }

  if constexpr (lean) {
    if (valid || padcol) {
#pragma unroll
      for (int q = 0; q < E; ++q) *dst_at(q) = valid ? v[q] : cx<T>{T(0), T(0)};
    }
  } else {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (valid || padcol) a.dst[base + (int64_t)(j + q * P) * a.s] = valid ? v[q] : cx<T>{T(0), T(0)};
    }
  }
}

}  // namespace ffcz
