// Edit coding around the correction loop (Alg. 1 edit bookkeeping, CompactEdits and
// QuantizeEdits of Sec. IV-B / IV-D, and their inverse for applying edits).
//
// Coordinates.  The spatial edits have one coordinate per real point (C order).
// The frequency edits have two per half-spectrum entry, Re then Im, entries in C
// order over rows of H + 1 entries; in the workspace those rows sit at the
// spectrum's padded pitch and plane.  A flag bit per coordinate says whether its
// edit is non-zero; flags are packed eight to a byte, coordinate 8 b + i in bit i
// of byte b (least significant bit first).  The non-zero edits are stored in
// coordinate order, each at the exclusive prefix count of the flags before it,
// as m-bit quantisation codes rint(v / step) (int32, half to even).
//
// Work split.  A wave takes 64 consecutive coordinates at a time (one lane each),
// so its ballot IS the 64-bit flag word of those coordinates, and mbcnt of the
// ballot is each lane's prefix inside the word.  A block owns kEditChunks
// consecutive words; wave w takes words w, w + 4, ... of them.  Two launches
// over the same blocks: the first counts each block's non-zero coordinates, a
// one-block scan turns the counts into block offsets, the second writes flags
// and codes.  The decoder runs the same walk over flag words instead of values.
#pragma once
#include "common.hpp"

namespace ffcz {

constexpr int kEditWaves = 4;                     // waves per block (256 lanes)
constexpr int kEditChunks = 32;                   // 64-coordinate words per block
constexpr int64_t kEditBlockCoords = 64 * kEditChunks;

// One coordinate set: the spatial edits (dense, C order) or the frequency edits
// (complex entries in the padded spectrum layout, Re/Im interleaved).
template <typename T>
struct EditSet {
  T* val;           // spatial: N values; frequency: the spectrum buffer as reals
  int64_t ncoord;   // N, or 2 M
  int32_t freq;     // 0 spatial, 1 frequency
  int32_t ncols;    // frequency: entries per row (H + 1)
  int64_t pitch;    // frequency: complex entries per row of the buffer
  int64_t plane;    // frequency: complex entries per plane of 2^lg_rpp rows
  int32_t lg_rpp;
  int32_t pad;
};

// Element offset (in T) of coordinate c of a set.
template <typename T>
__device__ __forceinline__ int64_t edit_offset(const EditSet<T>& s, int64_t c) {
  if (!s.freq) return c;
  const int64_t e = c >> 1;
  const int64_t r = e / s.ncols;
  const int64_t col = e - r * s.ncols;
  const int64_t addr = (r >> s.lg_rpp) * s.plane + (r & ((int64_t(1) << s.lg_rpp) - 1)) * s.pitch + col;
  return 2 * addr + (c & 1);
}

__device__ __forceinline__ int lane_prefix(unsigned long long m) {
  // set bits of m below this lane
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Block sum of per-wave counts through LDS, in wave order; returns every wave's
// exclusive offset in excl[w] and the total.
__device__ __forceinline__ unsigned long long block_wave_scan(unsigned long long mine, unsigned long long* lds,
                                                              unsigned long long* excl) {
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = mine;
  __syncthreads();
  unsigned long long run = 0;
#pragma unroll
  for (int i = 0; i < kEditWaves; ++i) {
    excl[i] = run;
    run += lds[i];
  }
  __syncthreads();
  return run;
}

// Pass 1 of CompactEdits: non-zero coordinates per block.
template <typename T>
__global__ void __launch_bounds__(64 * kEditWaves) edit_count_kernel(EditSet<T> s, unsigned long long* part) {
  __shared__ unsigned long long red[kEditWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kEditBlockCoords;
  unsigned long long cnt = 0;
#pragma unroll 4
  for (int it = w; it < kEditChunks; it += kEditWaves) {
    const int64_t c = c0 + (int64_t)it * 64 + lane;
    const bool nz = c < s.ncoord && s.val[edit_offset(s, c)] != T(0);
    cnt += (unsigned long long)__popcll(__ballot(nz));
  }
  if (lane == 0) red[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < kEditWaves; ++i) t += red[i];
    part[blockIdx.x] = t;
  }
}

// Exclusive scan of n block counts in place (one block of 1024 lanes, each lane
// a contiguous run); the total goes to *total.
__global__ void __launch_bounds__(1024) edit_scan_kernel(unsigned long long* part, int64_t n,
                                                         unsigned long long* total) {
  __shared__ unsigned long long red[16];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = (int64_t)t * per < n ? (int64_t)t * per : n;
  const int64_t hi = lo + per < n ? lo + per : n;
  unsigned long long mine = 0;
  for (int64_t i = lo; i < hi; ++i) mine += part[i];
  // inclusive scan over the lanes of the wave, then over the waves
  unsigned long long inc = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long o = __shfl_up(inc, off, 64);
    if ((t & 63) >= off) inc += o;
  }
  if ((t & 63) == 63) red[t >> 6] = inc;
  __syncthreads();
  unsigned long long wbase = 0;
  for (int i = 0; i < (t >> 6); ++i) wbase += red[i];
  unsigned long long run = wbase + inc - mine;
  for (int64_t i = lo; i < hi; ++i) {
    const unsigned long long v = part[i];
    part[i] = run;
    run += v;
  }
  if (t == 1023) *total = run;
}

// Status bits the coding kernels raise (OR-ed into one word).
constexpr unsigned kEditCodeRange = 1u;  // a code outside int32 (or a non-zero edit with a zero step)
constexpr unsigned kEditFlagCount = 2u;  // decoder: set flags and given code count disagree

// Pass 2 of CompactEdits fused with QuantizeEdits: flag words and codes.
template <typename T>
__global__ void __launch_bounds__(64 * kEditWaves) edit_write_kernel(EditSet<T> s, const unsigned long long* off,
                                                                     uint8_t* flags, int32_t* codes, double step,
                                                                     unsigned* status) {
  __shared__ unsigned long long red[kEditWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kEditBlockCoords;
  const int64_t nbytes = (s.ncoord + 7) >> 3;
  unsigned long long run = off[blockIdx.x];
  unsigned bad = 0;
  for (int base = 0; base < kEditChunks; base += kEditWaves) {
    const int it = base + w;
    const int64_t cw = c0 + (int64_t)it * 64;  // first coordinate of this wave's word
    const int64_t c = cw + lane;
    T v = T(0);
    if (c < s.ncoord) v = s.val[edit_offset(s, c)];
    const bool nz = v != T(0);
    const unsigned long long m = __ballot(nz);
    unsigned long long ex[kEditWaves];
    const unsigned long long tot = block_wave_scan((unsigned long long)__popcll(m), red, ex);
    if (nz) {
      const double q = step > 0.0 ? rint((double)v / step) : 0.0;
      if (!(step > 0.0) || !(fabs(q) < 2147483648.0)) bad |= kEditCodeRange;
      codes[run + ex[w] + lane_prefix(m)] = (int32_t)(fabs(q) < 2147483648.0 ? q : 0.0);
    }
    // the flag word: whole words as one 8-byte store, the last partial word byte by byte
    if (cw < s.ncoord) {
      const int64_t b0 = cw >> 3;
      if (b0 + 8 <= nbytes) {
        if (lane == 0) *reinterpret_cast<unsigned long long*>(flags + b0) = m;
      } else if (lane < 8 && b0 + lane < nbytes) {
        flags[b0 + lane] = (uint8_t)(m >> (8 * lane));
      }
    }
    run += tot;
  }
  if (bad) atomicOr(status, bad);
}

// Flag word i of a set (zero bits past the last coordinate).
__device__ __forceinline__ unsigned long long flag_word(const uint8_t* flags, int64_t ncoord, int64_t i) {
  const int64_t nbytes = (ncoord + 7) >> 3;
  const int64_t b0 = i * 8;
  if (b0 + 8 <= nbytes) return *reinterpret_cast<const unsigned long long*>(flags + b0);
  unsigned long long m = 0;
  for (int k = 0; k < 8 && b0 + k < nbytes; ++k) m |= (unsigned long long)flags[b0 + k] << (8 * k);
  return m;
}

// Decoder pass 1: set flags per block.
__global__ void __launch_bounds__(64 * kEditWaves) flag_count_kernel(const uint8_t* flags, int64_t ncoord,
                                                                     unsigned long long* part) {
  __shared__ unsigned long long red[kEditWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t w0 = (int64_t)blockIdx.x * kEditChunks;
  const int64_t nwords = (ncoord + 63) >> 6;
  unsigned long long cnt = 0;
  for (int it = w; it < kEditChunks; it += kEditWaves) {
    const int64_t i = w0 + it;
    if (i < nwords && lane == 0) {
      unsigned long long m = flag_word(flags, ncoord, i);
      const int64_t rem = ncoord - i * 64;
      if (rem < 64) m &= (1ull << rem) - 1ull;  // bits past the last coordinate do not count
      cnt += (unsigned long long)__popcll(m);
    }
  }
  if (lane == 0) red[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < kEditWaves; ++i) t += red[i];
    part[blockIdx.x] = t;
  }
}

// Decoder pass 2: dense dequantised edits, code * step at flagged coordinates and 0
// elsewhere, written as TO at the set's offsets (spatial: the output field; frequency:
// the spectrum buffer).  Codes past ncodes are never read (the flag count is checked).
template <typename TO>
__global__ void __launch_bounds__(64 * kEditWaves) edit_expand_kernel(EditSet<TO> s, const uint8_t* flags,
                                                                      const int32_t* codes, int64_t ncodes,
                                                                      const unsigned long long* off, double step,
                                                                      const unsigned long long* total,
                                                                      unsigned* status) {
  __shared__ unsigned long long red[kEditWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kEditBlockCoords;
  if (*total != (unsigned long long)ncodes) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, kEditFlagCount);
    return;
  }
  unsigned long long run = off[blockIdx.x];
  for (int base = 0; base < kEditChunks; base += kEditWaves) {
    const int it = base + w;
    const int64_t cw = c0 + (int64_t)it * 64;
    const int64_t c = cw + lane;
    unsigned long long m = 0;
    if (cw < s.ncoord) {
      m = flag_word(flags, s.ncoord, cw >> 6);
      const int64_t rem = s.ncoord - cw;
      if (rem < 64) m &= (1ull << rem) - 1ull;
    }
    unsigned long long ex[kEditWaves];
    const unsigned long long tot = block_wave_scan((unsigned long long)__popcll(m), red, ex);
    if (c < s.ncoord) {
      const bool set = (m >> lane) & 1ull;
      const int64_t pos = (int64_t)(run + ex[w]) + lane_prefix(m);
      const double v = set && pos < ncodes ? (double)codes[pos] * step : 0.0;
      s.val[edit_offset(s, c)] = (TO)v;
    }
    run += tot;
  }
}

// Dense copy of a coordinate set (the accumulators in coordinate order).
template <typename T>
__global__ void __launch_bounds__(256) edit_export_kernel(EditSet<T> s, T* out) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < s.ncoord) out[c] = s.val[edit_offset(s, c)];
}

// Fill n values of T with zero (the frequency accumulators before the loop; a kernel, so
// that a captured stream records no memset node).
template <typename T>
__global__ void __launch_bounds__(256) zero_fill_kernel(T* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = T(0);
}

}  // namespace ffcz
