// Device state, kernel argument blocks and pass modes shared by the kernels
// and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace ffcz {

// Loop state kept in the caller's workspace.  Written by one lane at a time
// (the set-up kernel or the per-round control kernel); read at the entry of
// every loop kernel.
struct DevState {
  // parameters: bounds, the shrunk s-bound, the check threshold and the shrunk f-bound
  double E, Ep, Delta, Dc, Dp, inv_n;
  int32_t max_iter, fixed, record_masks, pad0;
  // loop control
  int32_t done, round, converged, nonfinite_stop;
  uint32_t ticket, pad1;
  // counters
  unsigned long long nonfinite, s_guard, s_clipped_total;
  unsigned long long max_spatial_bits, max_spectral_bits, spectral_viol;
  // the margin mu in use (given, or derived on the device from x before the first pass)
  double mu;
  // violation counts of the first and of the last check (ctl_kernel), so the host reads one struct
  unsigned long long v_first, v_last;
  // the instance's data (device pointers): x, x_hat (or dL/dy), y (or dL/dx_hat)
  const void* px;
  const void* pxb;
  void* py;
  // the encoder's spatial shrink (its spectral shrink is mu)
  double mu_s;
  // pointwise bounds (ffcz_correct_bounds): E_n in the field's layout and dtype (null: the
  // scalar E), (D^Re_k, D^Im_k) pairs of the working type laid out as the spectrum; a bound b
  // gives the shrunk s-bound b fe, the check threshold b fc and the shrunk f-bound b fp
  const void* pE;
  const void* pD;
  double fe, fc, fp;
  int32_t disk;  // 1: |delta_k| <= D^Re_k (modulus), radial projection
  int32_t pad3;
};

enum ColMode : int {
  COL_FWD = 0,     // forward C2C along the strided axis
  COL_INV = 1,     // inverse C2C
  COL_XPASS = 2,   // forward, count + clip (+ f-mask), inverse; decides convergence
  COL_XBACK = 3,   // forward, multiply by recorded f-mask, inverse (adjoint)
  COL_VERIFY = 4,  // forward (FP64), max |Re|,|Im| and violation count; no store
  COL_FWD_NS = 5,  // forward, ignores the done flag (adjoint, verification)
  COL_INV_NS = 6,  // inverse, ignores the done flag (adjoint, decoder)
  COL_XEDIT = 7,   // COL_XPASS that also adds each clip displacement to the frequency edits
  COL_XUNDO = 8,   // forward and clip as COL_XPASS, then subtracts the displacement from the
                   // frequency edits (the check that ended the loop discards its clip); no store
  COL_XPASSP = 9,  // COL_XPASS against pointwise bounds (box on Re and Im, or the disk)
  COL_VERIFYP = 10 // COL_VERIFY against pointwise bounds: max ratio to the bound, violations
};

enum RowMode : int {
  ROW_INIT = 0,    // eps0 = x_hat - x (FP64), guard clip, R2C
  ROW_LOOP = 1,    // C2R, 1/N, s-clip (+ s-mask), R2C
  ROW_FINAL = 2,   // C2R, 1/n_last, y = x + eps in FP64, closing clamp, store y
  ROW_VERIFY = 3,  // d = y - x in FP64, max |d|, FP64 R2C
  ROW_BINIT = 4,   // g * s-mask, R2C        (adjoint)
  ROW_BLOOP = 5,   // C2R, 1/N, g * s-mask, R2C (adjoint)
  ROW_BFINAL = 6,  // C2R, 1/N, g * s-mask, store (adjoint)
  ROW_FINALV = 7,  // FP64 fields: ROW_FINAL, then d = y - x from the stored y: max |d|, FP64 R2C (the
                   // last-axis pass of the verification, without re-reading x and y)
  ROW_INITE = 8,   // ROW_INIT that also stores each guard-clip displacement as the first spatial edit
  ROW_LOOPE = 9,   // ROW_LOOP that also adds each s-clip displacement to the spatial edits
  ROW_DECODE = 10, // C2R, 1/N, y = x_hat + s + eps summed in FP64 and rounded once (decoder; s in py)
  ROW_INITP = 11,  // ROW_INIT with a spatial bound per point
  ROW_LOOPP = 12,  // ROW_LOOP with a spatial bound per point
  ROW_FINALP = 13, // ROW_FINAL with a spatial bound per point (closing clamp against E_n)
  ROW_VERIFYP = 14 // ROW_VERIFY keeping max |y_n - x_n| / E_n instead of max |y_n - x_n|
};

template <typename T>
struct ColArgs {
  const cx<T>* src;
  cx<T>* dst;
  int64_t so;      // stride between outer indices (complex entries)
  int64_t s;       // stride along the transformed axis
  int32_t ncols;   // valid contiguous columns
  int32_t ncols_pad;  // columns of the padded row: those past ncols are stored as zeros
  int32_t ncb;     // column blocks per outer index
  int64_t outer_per_inst;  // outer indices per instance (instance = outer / outer_per_inst)
  const cx<T>* tw; // stage twiddles of this length
  DevState* st;    // per-instance loop state
  unsigned long long* part;  // one partial result per block (count; verification: + max at part_stride)
  int64_t part_stride;
  // f-masks (forward record / adjoint read)
  uint8_t* fmask;      // forward: base of the f-mask region; adjoint: Re plane of block k
  int64_t f_plane;     // bytes per Re (or Im) plane
  int64_t f_row_bytes; // bytes per half-spectrum row
  int64_t mrow_i;      // mask row = i * mrow_i + outer * mrow_o
  int64_t mrow_o;
  // frequency edits (COL_XEDIT / COL_XUNDO): same layout as the spectrum the pass transforms
  cx<T>* fedit;
  // pointwise spectral bounds (COL_XPASSP / COL_VERIFYP): (Re, Im) pairs of floats (bnd_dbl 0)
  // or doubles at bnd_so * outer + column + bnd_s * i, the transformed spectrum's own layout
  // in the loop, the working-type spectrum's layout in the FP64 verification
  const void* bnd;
  int64_t bnd_so, bnd_s;
  int32_t bnd_dbl;
  // neighbouring tiles that share 128-byte lines (1: none); the grid holds a multiple of it per
  // outer index and the kernel runs each such group on one XCD (xcd_tile)
  int32_t xcd_k;
};

// Logical tile of physical block p.  Blocks are dealt round-robin to the 8 XCDs, each with its
// own L2.  When a tile is narrower than a 128-byte line, k neighbouring tiles read parts of the
// same lines; the k tiles of an aligned run go to physical blocks x, x + 8, ..., x + 8 (k - 1)
// of a group of 8 k, which land on one XCD at about the same time, so each line is fetched into
// that L2 once.  A ragged last group keeps the plain order.  A permutation: every tile runs once.
__device__ __forceinline__ int64_t xcd_tile(int64_t p, int64_t n, int k) {
  if (k <= 1) return p;
  const int64_t G = 8 * (int64_t)k;
  const int64_t g = p / G;
  if ((g + 1) * G > n) return p;
  const int64_t r = p - g * G;
  return g * G + (int64_t)k * (r & 7) + (r >> 3);
}

template <typename T, typename TIO>
struct RowArgs {
  const cx<T>* src;
  cx<T>* dst;
  int64_t pitch;          // complex entries per spectrum row
  int64_t rows_per_inst;  // rows of one instance (spectrum rows are contiguous across instances)
  int64_t bpi;            // blocks per instance
  const cx<T>* tw;        // stage twiddles of length H followed by H R2C twiddles
  DevState* st;           // per-instance loop state (also holds the instance's data pointers)
  unsigned long long* part;  // one partial result per block (clip count or max bits)
  uint32_t* smask;   // forward: base of the s-mask region; adjoint: s-mask plane to apply
  int64_t s_plane;   // uint32 words per s-mask plane
  int32_t s_row_w32; // uint32 words per s-mask row
  int32_t pad;
  int64_t plane;     // complex entries per plane of rows (src / dst spectra)
  int32_t lg_rpp;    // log2 of the rows per plane
  int32_t pad2;
  // source spectrum layout (complex entries per row / plane); differs from pitch / plane
  // only where a pass reads one precision and writes another (ROW_FINALV)
  int64_t spitch;
  int64_t splane;
  // spatial edits (ROW_INITE / ROW_LOOPE): one value per real point of the instance, C order
  T* sedit;
};

// FP64 bound -> working type, rounded toward zero (a tighter bound in FP32).
template <typename T>
__device__ __forceinline__ T to_t(double v);
template <>
__device__ __forceinline__ float to_t<float>(double v) { return __double2float_rz(v); }
template <>
__device__ __forceinline__ double to_t<double>(double v) { return v; }

// Clip to [-b, b] (b >= 0, v finite).  FP32: one v_med3_f32, the median of (v, -b, b), which
// returns one of its inputs, so an unclipped value comes back unchanged.
template <typename T>
__device__ __forceinline__ T clipv(T v, T b) { return v > b ? b : (v < -b ? -b : v); }
template <>
__device__ __forceinline__ float clipv<float>(float v, float b) { return __builtin_amdgcn_fmed3f(v, -b, b); }

// Columns per block: 128-byte rows, halved until the tile fits in 128 KiB of LDS.
template <typename T>
__host__ __device__ constexpr int pick_C(int L) {
  int c = 128 / (int)sizeof(cx<T>);
  while (c > 1 && (long)c * L * (long)sizeof(cx<T>) > 128 * 1024) c /= 2;
  return c;
}
// Elements per lane of the last-axis transforms (radix-16 stages from H = 64 on).
__host__ __device__ constexpr int pick_E_row(int H) { return H >= 64 ? 16 : pick_E(H); }

// LDS rows of the last-axis passes.  Lanes run rows-fastest (ROWS rows x 64/ROWS
// indices per wave) and rows sit an odd pitch H + 1 apart, which keeps a wave's
// accesses on distinct banks while a wave spans many rows.  With few rows per
// block (long rows) the indices of one row collide instead, so for those shapes
// entry i of a row moves to i + (i >> 5) (one skip per 32 entries) and the pitch
// takes a pad chosen by a model of the kernel's LDS access patterns (the
// compute-mapping reads and writes, the Stockham exchanges, the R2C unpack, the
// row-major loads and stores): the worst slot load drops from 8-32 lanes to 3
// (8-byte entries) or 5-6 (16-byte).  Shapes whose odd pitch stays below four
// times the unavoidable 2 (4) lanes per slot keep it: there the skew's index
// arithmetic costs more than it saves (measured on the 256-entry rows).
__host__ __device__ constexpr int row_lds_pad(int H, int R, int E, int S) {
  if (H == 512 && R == 2 && E == 16 && S == 16) return 0;
  if (H == 512 && R == 4 && E == 16 && S == 16) return 6;
  if (H == 512 && R == 8 && E == 16 && S == 8) return 8;
  if (H == 1024 && R == 1 && E == 16 && S == 16) return 0;
  if (H == 1024 && R == 2 && E == 8 && S == 16) return 7;
  if (H == 1024 && R == 2 && E == 16 && S == 8) return 15;
  if (H == 1024 && R == 2 && E == 16 && S == 16) return 0;
  if (H == 1024 && R == 4 && E == 8 && S == 8) return 12;
  if (H == 1024 && R == 4 && E == 8 && S == 16) return 2;
  if (H == 1024 && R == 4 && E == 16 && S == 8) return 5;
  if (H == 1024 && R == 4 && E == 16 && S == 16) return 4;
  if (H == 1024 && R == 8 && E == 8 && S == 8) return 2;
  if (H == 1024 && R == 8 && E == 16 && S == 8) return 2;
  if (H == 2048 && R == 1 && E == 16 && S == 8) return 0;
  if (H == 2048 && R == 1 && E == 16 && S == 16) return 0;
  if (H == 2048 && R == 1 && E == 8 && S == 8) return 0;
  if (H == 2048 && R == 1 && E == 8 && S == 16) return 0;
  if (H == 2048 && R == 2 && E == 8 && S == 8) return 7;
  if (H == 2048 && R == 2 && E == 8 && S == 16) return 7;
  if (H == 2048 && R == 2 && E == 16 && S == 8) return 15;
  if (H == 2048 && R == 2 && E == 16 && S == 16) return 0;
  if (H == 2048 && R == 4 && E == 8 && S == 8) return 5;
  if (H == 2048 && R == 4 && E == 8 && S == 16) return 2;
  if (H == 2048 && R == 4 && E == 16 && S == 8) return 5;
  if (H == 2048 && R == 8 && E == 16 && S == 8) return 2;
  return -1;  // no skew: odd pitch
}
__host__ __device__ constexpr int row_lds_shift(int H, int R, int E, int S) {
  return row_lds_pad(H, R, E, S) >= 0 ? 5 : 0;
}
template <typename T>
__host__ __device__ constexpr int row_lds_pitch(int H, int R, int E) {
  return row_lds_pad(H, R, E, (int)sizeof(cx<T>)) >= 0
             ? H + (H >> 5) + 1 + row_lds_pad(H, R, E, (int)sizeof(cx<T>))
             : H + 1;
}

// LDS bytes of a last-axis block: its rows at their pitch, the stage and R2C
// twiddle tables, per-wave partial words and the rows' mask words.
template <typename T>
__host__ __device__ constexpr long row_lds_bytes(int H, int R, int E) {
  const long cs = (long)sizeof(cx<T>);
  const int P = H / E > 0 ? H / E : 1;
  const long nw = (R * P + 63) / 64;
  const long sw = 2 * (H >= 32 ? H / 32 : 1);
  return R * (long)row_lds_pitch<T>(H, R, E) * cs + (long)(host_twsize(H, E) + H) * cs + 16 * nw + 4 * R * sw;
}
// Rows per block of a last-axis plan with E elements per lane: up to 64 (one row
// per lane of a wave at a time), at most 1024 lanes, and at most 78 KiB of LDS,
// so that two blocks share a CU (the twiddle tables alone take 16 KiB at 1024
// FP32 entries; counting only the rows left one block per CU there).
template <typename T>
__host__ __device__ constexpr int rows_for_E(int H, int E) {
  const int P = H / E > 0 ? H / E : 1;
  int r = 64;
  while (r > 1 && (r * P > 1024 || row_lds_bytes<T>(H, r, E) > 78 * 1024)) r /= 2;
  return r;
}
template <typename T>
__host__ __device__ constexpr int pick_rows(int H) { return rows_for_E<T>(H, pick_E_row(H)); }

// Plans the tuner chooses between.  Column passes: variant 1 halves the tile
// width.  Last-axis passes: variant 1 halves the rows per block; variant 2
// uses radix-8 stages (8 elements per lane, twice the lanes per row) where the
// default is radix 16; variant 3 is the FP32 loop pass of 256-entry rows with
// lanes index-fastest and rows moved straight between HBM and registers
// (elsewhere it runs variant 1, whose rows per block it shares).  Variants 0 and
// 1 compute identical bits; variants 2 and 3 round differently (other stages,
// other fused multiply-adds).
constexpr int kColVariants = 2;
constexpr int kRowVariants = 4;
template <typename T>
__host__ __device__ constexpr int tile_cols(int L, int v) {
  return (pick_C<T>(L) >> v) < 1 ? 1 : (pick_C<T>(L) >> v);
}
// Elements per lane of a last-axis plan.
__host__ __device__ constexpr int row_E(int H, int v) { return (v == 2 && pick_E_row(H) == 16) ? 8 : pick_E_row(H); }

template <typename T>
__host__ __device__ constexpr int tile_rows(int H, int v) {
  if (v == 2) return rows_for_E<T>(H, row_E(H, 2));
  if (v == 3) v = 1;
  return (pick_rows<T>(H) >> v) < 1 ? 1 : (pick_rows<T>(H) >> v);
}

}  // namespace ffcz
