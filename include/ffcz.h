/*
 * ffcz.h -- C ABI of the MI355X (gfx950) dual-domain error correction.
 *
 * The library corrects a base compressor's reconstruction x_hat of a field x
 * so that the error eps = y - x satisfies both bounds of Eq. 2 of the FFCz
 * paper (Sec. IV-A):
 *     |eps_n| <= E                                   for every point n,
 *     |Re delta_k| <= Delta and |Im delta_k| <= Delta for every frequency k,
 * where delta = DFT(eps) is the unnormalised forward DFT of Eq. 1 (sign -i).
 * It runs the alternating projection of Alg. 1 (Sec. IV-B): forward FFT,
 * violation count (CheckConvergence), clip of Re and Im (ProjectOntoFCube),
 * inverse FFT, clip of eps (ProjectOntoSCube), until no coefficient violates.
 *
 * Conventions shared by every entry point
 *  - Every data pointer is a DEVICE pointer, 16-byte aligned, owned by the
 *    caller.  The library allocates no device memory: scratch comes from the
 *    caller's workspace (ffcz_correct_noalloc: from a fixed device array that
 *    the library holds per GPU).  Fields are C-ordered (last axis contiguous); the
 *    real-to-complex half-spectrum runs along the last axis.
 *  - dtype selects the storage type of x, x_hat, y and gradients: FFCZ_F32
 *    (float) or FFCZ_F64 (double).  FFCZ_F32 runs its transforms in FP32 with
 *    twiddle tables evaluated in FP64 and rounded once; the output clamp and
 *    the bound verification always run in FP64.
 *  - Shapes: 1 <= ndim <= 3, every extent >= 1; unit extents are squeezed
 *    away.  Fields of two or three remaining axes need every extent a power of
 *    two, the last one between 2 and 4096 and the others at most 2048 (FP32) /
 *    1024 (FP64).  A field with one remaining axis takes any length up to 2^19
 *    (a single point included): powers of two from 2 to 4096 run on the same
 *    passes as 2D/3D fields, every other length on the 1D signal path of
 *    ffcz_correct_batched (four-step or Bluestein DFT), which records no masks
 *    and no per-check counts.  Violation counts refer to the half-spectrum of
 *    the squeezed shape.
 *  - stream is a hipStream_t (NULL = the null stream).  Work is stream-ordered.
 *  - Return value: an ffcz_status.  Negative values are errors (the output is
 *    unspecified); ffcz_last_error() then describes the cause.
 *  - Bounds are shrunk by (1 - mu) for the projections and checked unshrunk
 *    (the m = 16 shrink of Sec. IV-B, mu = 2^-16 by default), which makes the
 *    loop terminate.
 */
#ifndef FFCZ_H
#define FFCZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FFCZ_F32 = 0, FFCZ_F64 = 1 } ffcz_dtype;

typedef enum {
  FFCZ_OK = 0,             /* converged; FP64 re-verification passed (if run)       */
  FFCZ_NOT_CONVERGED = 1,  /* max_iter rounds ran; y holds the last iterate (in S)   */
  FFCZ_VERIFY_FAILED = 2,  /* converged but the FP64 re-check of the output failed   */
  FFCZ_E_INVALID = -1,     /* bad scalar argument or null pointer                    */
  FFCZ_E_SHAPE = -2,       /* unsupported ndim / extent                              */
  FFCZ_E_WORKSPACE = -3,   /* workspace too small or misaligned                      */
  FFCZ_E_NONFINITE = -4,   /* x or x_hat holds NaN or Inf                            */
  FFCZ_E_HIP = -5          /* a HIP runtime call failed                              */
} ffcz_status;

typedef struct {
  /* Relative shrink mu of both bounds for the projections.  0 selects the
   * default: 2^-16 for FFCZ_F64; for FFCZ_F32 the value of
   * ffcz_suggest_margin() (room for the FP32 rounding of the output).
   * FP64: the check counts |Re|,|Im| > Delta and the projections clip to
   * E (1 - mu) and Delta (1 - mu).  FP32: the check counts |Re|,|Im| >
   * Delta (1 - mu) and the f-projection clips to Delta (1 - 2 mu), so that
   * rounding y to FP32 cannot lift an accepted coefficient above Delta. */
  double margin_rel;
  /* 1: run exactly max_iter projection blocks whatever the check says (the
   * map x_hat -> y is then piecewise linear; used for differentiation). */
  int32_t fixed_iterations;
  /* 1 (default): FP64 re-verification of both bounds on the output. */
  int32_t verify_fp64;
  /* Optional device buffer of ffcz_mask_bytes(ndim, shape, max_iter) bytes that
   * receives the clip keep-masks (layout documented at ffcz_mask_bytes). */
  void* masks_out;
  /* Optional device int64 array of max_iter + 1 entries: violation count of
   * every check (entry k = check after k projection blocks; unused entries 0). */
  int64_t* viol_per_round;
  /* Rounds enqueued between two host polls of the device done-flag (0 = 4). */
  int32_t graph_chunk;
  /* 1 (default): the chunk of rounds between two polls is captured once in a
   * hipGraph (cached per shape, workspace and output pointers) and replayed on
   * the caller's stream; 0: plain launches.  Ignored while profiling. */
  int32_t use_graph;
  /* Batched 1D members whose power-of-two work length Mc (Mc = L for a
   * power-of-two L >= 4, else the Bluestein length >= L + floor(L/2)) is at least
   * 2^tiled_1d_lg run as tiled passes, many blocks per signal, with the rounds
   * driven by the host; shorter ones run one block per signal for the whole
   * correction.  Values below 12 count as 12; above 20 keep every 1D member on
   * one block.  0 (default): work lengths below 2^12 run one block per signal,
   * above 2^16 tiled, and each length class between takes the plan tuner's
   * decision (ffcz_set_tuning): on its first use on a device architecture (per
   * data type and power-of-two bucket of the class's signal count) both forms
   * run three fixed rounds on the call's own members, before the correction,
   * and the faster is kept; with tuning off, classes from 2^15 run tiled.
   * Both forms give bit-identical results. */
  int32_t tiled_1d_lg;
  /* 1 (default): a 1D member that runs on one block keeps its work buffer in
   * that block's LDS when it fits (FP32 work length up to 2^14, FP64 up to
   * 2^13); 0: in the workspace.  Both give bit-identical results. */
  int32_t resident_1d;
} ffcz_options;

typedef struct {               /* host struct filled on return */
  int32_t rounds;              /* completed projection blocks                     */
  int32_t converged;           /* 1 if the last check found no violation          */
  int64_t f_viol_initial;      /* violations at the first check                   */
  int64_t f_viol_final;        /* violations at the last check                    */
  int64_t s_clipped_total;     /* spatial clips summed over all blocks             */
  int64_t s_guard;             /* initial errors clipped into the shrunk s-cube    */
  int64_t nonfinite;           /* non-finite inputs found                          */
  double max_spatial_err;      /* FP64 max |y - x| (verification)                  */
  double max_spectral_err;     /* FP64 max(|Re|,|Im|) of DFT(y - x)               */
  int64_t spectral_viol;       /* coefficients above Delta in the verification    */
  double margin_used;          /* mu actually used                                */
  int32_t status;              /* this instance's own ffcz_status                 */
  int32_t reserved;            /* 0                                               */
} ffcz_stats;

/* Library version (major*10000 + minor*100 + patch). */
int32_t ffcz_version(void);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* ffcz_last_error(void);

/* Fill *opts with the defaults described in ffcz_options. */
void ffcz_default_options(ffcz_options* opts);

/* Workspace bytes ffcz_correct / ffcz_correct_backward / ffcz_suggest_margin
 * need for this dtype, shape and round cap (a negative cap counts as 0; the
 * calls themselves reject it).  0 if the shape is unsupported.
 * Holds two half-spectrum buffers, the twiddle tables and the loop state. */
size_t ffcz_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter);

/* Bytes of the clip keep-mask record for `rounds` projection blocks.
 * Layout (little-endian 64-bit words, bit b of a word = element 64*w + b of
 * its row; a bit is 1 iff the projection left that component unchanged):
 *   rows_s = N / n_last rows of ceil(n_last/64) words          ("s-mask"),
 *   rows_f = N / n_last rows of ceil((n_last/2+1)/64) words    ("f-mask"),
 *   [s-mask 0 (guard)] [s-mask 1] ... [s-mask rounds]
 *   [f-mask Re 1][f-mask Im 1] ... [f-mask Re rounds][f-mask Im rounds]
 * where the shape is the squeezed one and f rows run over the half-spectrum. */
size_t ffcz_mask_bytes(int32_t ndim, const int64_t* shape, int32_t rounds);

/* Suggested shrink mu for an FP32 output (FP64 outputs: 2^-16).  Rounding
 * y = x + eps to FP32 perturbs every spectral component by about
 * sigma * sqrt(N/2) with sigma^2 = mean(ulp(x)^2)/12; mu keeps eight of these
 * inside the shrunk f-cube: mu = max(2^-16, 8 sigma sqrt(N/2) / Delta),
 * capped at 0.5.  Reads x (device) once; blocks until *mu_out is written.
 * The device reduction needs scratch: workspace (256-byte aligned) holds at
 * least 1025 doubles (any ffcz_workspace_bytes() size does), and the result
 * comes back through mu_out with a status as return value, so that the
 * library allocates nothing.  Returns FFCZ_E_SHAPE / FFCZ_E_INVALID /
 * FFCZ_E_WORKSPACE for an unsupported shape, bad argument or short workspace. */
int32_t ffcz_suggest_margin(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_orig,
                            double delta_f, void* workspace, size_t workspace_bytes, void* stream,
                            double* mu_out);

/* Alg. 1 on one field.
 *   x_orig  original data x (device, dtype, shape)
 *   x_base  base reconstruction x_hat (device; may alias x_out, not x_orig)
 *   x_out   corrected y (device)
 *   eps_s   spatial bound E (>= 0, finite)
 *   delta_f spectral bound Delta on Re and Im (>= 0, finite)
 *   max_iter cap on projection blocks (>= 0)
 *   opts    NULL for defaults
 *   workspace / workspace_bytes  device scratch of ffcz_workspace_bytes() bytes
 *   stats   NULL or a host struct filled on return
 * The call blocks on the host once per graph_chunk rounds to read the device
 * done-flag, and at the end for the statistics and the status.  With
 * fixed_iterations = 1, stats = NULL and verify_fp64 = 0 nothing is reported,
 * so the call is fully asynchronous (no host synchronisation) and returns
 * FFCZ_OK once the work is enqueued; non-finite input is then not detected
 * (its entries are taken as zero error). */
int32_t ffcz_correct(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_orig,
                     const void* x_base, void* x_out, double eps_s, double delta_f,
                     int32_t max_iter, const ffcz_options* opts, void* workspace,
                     size_t workspace_bytes, void* stream, ffcz_stats* stats);

/* Bytes of the fixed device scratch array behind ffcz_correct_noalloc (64 MiB). */
#define FFCZ_NOALLOC_SCRATCH_BYTES (64u << 20)

/* ffcz_correct for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same correction, with the workspace taken from a fixed device array of
 * FFCZ_NOALLOC_SCRATCH_BYTES bytes that the library holds, one copy per GPU,
 * from the first call on that GPU until the process ends.  The call allocates
 * nothing (no hipMalloc, no pinned staging, no graph instantiation): the
 * rounds run as plain launches and the tile plans come from the tuning table
 * or the defaults (nothing is timed).
 *   Arguments and results as ffcz_correct, without workspace / workspace_bytes.
 *   Shapes: fields that run on the passes of 2D/3D fields (every remaining
 *   extent a power of two, as documented above); other 1D lengths return
 *   FFCZ_E_SHAPE.  A shape and round cap needing more than
 *   FFCZ_NOALLOC_SCRATCH_BYTES of workspace (ffcz_workspace_bytes) returns
 *   FFCZ_E_WORKSPACE (for example 128^3 FP32 needs about 21 MB, 256^3 FP32
 *   about 151 MB: refused).
 *   The current device (hipGetDevice) must be the one holding x_orig, x_base,
 *   x_out and the stream's work.
 *   Every call on one GPU uses that GPU's single array and leaves the last
 *   call's contents in it (the call sets up whatever must start at zero):
 *   calls that overlap on one GPU -- from two host threads, or on two streams
 *   not ordered with each other -- race on it and give undefined results. */
int32_t ffcz_correct_noalloc(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_orig,
                             const void* x_base, void* x_out, double eps_s, double delta_f,
                             int32_t max_iter, const ffcz_options* opts, void* stream, ffcz_stats* stats);

/* ---------------------------------------------------------------------------
 * Edit coding (Alg. 1 edit bookkeeping; CompactEdits and QuantizeEdits of
 * Sec. IV-B and IV-D; applying edits, Sec. IV-B).
 *
 * The encoder runs the correction loop while summing every displacement of
 * ProjectOntoSCube into the spatial edits s (the guard clip that puts the
 * initial error inside the s-cube counts as the first) and every displacement
 * of ProjectOntoFCube into the frequency edits f (a half-spectrum), so that
 * eps_final = (x_hat - x) + s + IFFT(f).  The clip of the check that ends the
 * loop never reaches the iterate and is not counted.  It then codes both:
 *  - coordinates: s has N (the field's points, C order); f has 2 M, the Re and
 *    Im parts of the M half-spectrum entries of the squeezed shape, entries in
 *    C order, Re before Im;
 *  - flags: bit i of byte b is set iff coordinate 8 b + i has a non-zero edit
 *    (ceil(N / 8) and ceil(2 M / 8) bytes);
 *  - codes: int32 rint(v / step), half to even, of the non-zero edits in
 *    coordinate order (at the exclusive prefix count of the flags), with
 *    step_s = 2 E 2^-m and step_f = 2 Delta 2^-m (each cube side cut into 2^m
 *    steps; m = 16 in the paper).
 * Shrinks: the paper shrinks both cubes by 2^-m so that dequantised edits stay
 * inside.  The quantisation error of one domain also reaches the other through
 * the transform, and the decoder rounds its output with no clamp, so by
 * default the loop runs with q = safety 2^-m (safety 4) and
 *   mu_f = max(q, output-rounding margin of ffcz_correct),
 *   mu_s = q + spacing(max|x| + E) / E     (one output ulp),
 * checking |Re|,|Im| > Delta (1 - mu_f), clipping to Delta (1 - 2 mu_f) and to
 * E (1 - mu_s).  The decoded output is meant to be re-verified, not trusted. */

typedef struct {
  int32_t m;            /* code length (0: 16), at most 30                            */
  int32_t pad;
  double safety;        /* q = safety 2^-m (0: 4)                                     */
  double mu_s;          /* given shrinks (both or neither; 0: derived as above)       */
  double mu_f;
  void* y_out;          /* nullable device field: also y = x + eps with the closing
                           clamp of ffcz_correct, FP64-verified if opts asks for it  */
  void* spat_edits_out; /* nullable device buffer: s, N values of dtype              */
  void* freq_edits_out; /* nullable device buffer: f, 2 M values of dtype (Re, Im)   */
} ffcz_encode_options;

typedef struct {        /* host struct filled on return */
  ffcz_stats loop;      /* the loop's statistics (verification fields: NaN without y_out) */
  int64_t nnz_s;        /* spatial codes written (= set spatial flags)    */
  int64_t nnz_f;        /* frequency codes written                        */
  double step_s;        /* 2 E 2^-m                                       */
  double step_f;        /* 2 Delta 2^-m                                   */
  double mu_s;          /* shrinks in use                                 */
  double mu_f;
  int32_t m;
  int32_t status;
} ffcz_encode_stats;

/* Fill *o with the defaults (m = 16, safety 4, derived shrinks, no extra outputs). */
void ffcz_default_encode_options(ffcz_encode_options* o);

/* Workspace bytes of ffcz_encode and ffcz_decode (the correction's workspace,
 * both accumulators and the coding kernels' block offsets); 0 if unsupported. */
size_t ffcz_encode_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter);

/* Alg. 1 with edit bookkeeping, CompactEdits and QuantizeEdits (lossless
 * coding of the codes aside).
 *   x_orig, x_base, eps_s, delta_f, max_iter, opts: as ffcz_correct (shapes
 *     that run on the multidimensional passes only: every remaining extent a
 *     power of two; other 1D lengths give FFCZ_E_SHAPE)
 *   eopts       NULL for defaults
 *   spat_flags  device, ceil(N / 8) bytes      spat_codes  device int32[N]
 *   freq_flags  device, ceil(2 M / 8) bytes    freq_codes  device int32[2 M]
 *     (codes: room for the worst case; the counts come back in stats)
 *   workspace   ffcz_encode_workspace_bytes() bytes, 256-byte aligned
 *   stats       NULL or a host struct filled on return
 * Returns the loop's status (FFCZ_NOT_CONVERGED: the edits describe the last
 * iterate), FFCZ_E_INVALID if a code does not fit int32.  Blocks until the
 * code counts are known. */
int32_t ffcz_encode(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_orig, const void* x_base,
                    double eps_s, double delta_f, int32_t max_iter, const ffcz_options* opts,
                    const ffcz_encode_options* eopts, void* spat_flags, int32_t* spat_codes, void* freq_flags,
                    int32_t* freq_codes, void* workspace, size_t workspace_bytes, void* stream,
                    ffcz_encode_stats* stats);

/* Applying edits (Sec. IV-B): y = x_hat + s + IFFT(f), with s and f
 * dequantised from the flags and codes ffcz_encode wrote (code * step), the
 * sum formed in FP64 and rounded once to dtype.  x_base is the base
 * reconstruction the encoder was given; y must not alias it.  nnz_s / nnz_f:
 * the number of codes in each set, checked against the set flags (a mismatch
 * returns FFCZ_E_INVALID and leaves y unspecified).  Blocks until that check
 * is read back. */
int32_t ffcz_decode(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_base,
                    const void* spat_flags, const int32_t* spat_codes, int64_t nnz_s, const void* freq_flags,
                    const int32_t* freq_codes, int64_t nnz_f, double step_s, double step_f, void* y_out,
                    void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Generalised bounds (the footnote to Eq. 2, Sec. IV-A; Sec. V-B, Observation 4).
 *
 * Pointwise bounds replace the scalars point by point and entry by entry:
 * |eps_n| <= E_n, |Re delta_k| <= D^Re_k and |Im delta_k| <= D^Im_k, or with
 * disk = 1 |delta_k| <= D_k (the modulus, projected radially; D_k taken from
 * delta_re).  The loop, margins and verification are those of ffcz_correct,
 * entry by entry: FP64 output checks D_k and projects onto D_k (1 - mu) and
 * E_n (1 - mu); FP32 output checks D_k (1 - mu) and projects onto
 * D_k (1 - 2 mu), with the FP32 margin rule of ffcz_suggest_margin applied to
 * Delta = min_k D_k (times sqrt 2 for the disk).  Spectral bound arrays must
 * satisfy D_{-k} = D_k where the half-spectrum holds both entries (the k_z = 0
 * and Nyquist planes), as the bound of a real field's error does. */
typedef struct {
  const void* eps_s;     /* nullable device array: E_n, N values of dtype, C order
                            (NULL: the scalar eps_s of the call)                    */
  const void* delta_re;  /* nullable device array: D^Re_k (the disk's D_k), M values
                            of dtype, half-spectrum in C order (NULL: delta_f)      */
  const void* delta_im;  /* nullable: D^Im_k (NULL: delta_re, or delta_f)           */
  int32_t disk;          /* 1: bound the modulus by delta_re (delta_im unused)      */
  int32_t pad;
} ffcz_bounds;

/* Workspace bytes of ffcz_correct_bounds and ffcz_power_spectrum_bounds; 0 if unsupported. */
size_t ffcz_bounds_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter);

/* ffcz_correct with pointwise bounds (arrays in bnd, scalars eps_s / delta_f
 * where an array is NULL).  Shapes that run on the multidimensional passes
 * (every remaining extent a power of two); no masks (opts->masks_out must be
 * NULL).  Bound arrays with a negative or non-finite entry return
 * FFCZ_E_INVALID before the loop.  In the statistics, max_spatial_err is the
 * largest |y_n - x_n| / E_n and max_spectral_err the largest ratio of a part
 * (box) or of the modulus (disk) to its bound, both <= 1 on success (0 / 0
 * counts as 0).  Other arguments and results as ffcz_correct. */
int32_t ffcz_correct_bounds(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_orig,
                            const void* x_base, void* x_out, double eps_s, double delta_f,
                            const ffcz_bounds* bounds, int32_t max_iter, const ffcz_options* opts,
                            void* workspace, size_t workspace_bytes, void* stream, ffcz_stats* stats);

/* Relative power-spectrum bound (Sec. V-B, Observation 4): the pointwise
 * spectral bound D_k (written to delta_out, M values of dtype, half-spectrum
 * C order) that keeps every shell of the power spectrum within a relative
 * error rho for any error inside the bounds.  Shell b = rint(|k|) with |k| from
 * the signed integer frequencies; P_b = sum w_k |X_k|^2 over the shell (w_k = 2
 * for interior last-axis entries, 1 at k_z = 0 and at the Nyquist plane), with
 * X the FP64 DFT of x.  With S_b = sum w_k |X_k| and W_b = sum w_k, every entry
 * of shell b gets the largest D with 2 sqrt2 D S_b + 2 D^2 W_b <= rho P_b (box:
 * |Re|, |Im| <= D) or 2 D S_b + D^2 W_b <= rho P_b (disk = 1: |delta| <= D),
 * rounded toward zero in FP32.  The shell sums use atomic additions, so the
 * last bit of D can differ between calls.  Asynchronous on stream. */
int32_t ffcz_power_spectrum_bounds(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x_orig,
                                   double rho, int32_t disk, void* delta_out, void* workspace,
                                   size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Lossless coding of the edit streams (Alg. 1, LosslesslyCompressEdits;
 * Sec. IV-B, IV-D): Huffman coding of a stream of symbols -- the flag bytes
 * (width 1, unsigned) or the int32 codes (width 4) that ffcz_encode writes.
 * The symbols are counted blockwise into a global frequency table over
 * [min, max]; the code merges the two lightest nodes, ties going to the node
 * created first (leaves in symbol order, then merged nodes in turn); codes
 * longer than 32 bits halve every count ((c + 1) / 2) and rebuild; canonical
 * codes (by length, then value) are written most significant bit first into
 * 32-bit words filled from their top bit, with the bit offset of every 256th
 * symbol kept so that decoding runs one lane per 256 symbols.  The paper
 * follows this stage with ZSTD, a third-party compressor not part of this
 * library.
 * Stream (device bytes): a 64-byte header (magic "FHUF", width, symbol
 * count, smallest symbol, alphabet size, bit count, chunk count), the code
 * lengths (one byte per alphabet entry, padded to 16), the chunk offsets
 * (uint64), the 32-bit words. */
typedef struct {
  int64_t nsym;      /* symbols in the stream                                  */
  int64_t lo;        /* smallest symbol                                        */
  int64_t nalpha;    /* alphabet size: largest - smallest + 1 (at most 2^24)   */
  size_t ws_bytes;   /* workspace of ffcz_huffman_encode / ffcz_huffman_decode */
  size_t out_bytes;  /* output bytes that always suffice (32 bits a symbol)    */
} ffcz_huffman_sizes;

/* Workspace bytes for a stream of nsym symbols over an alphabet of nalpha
 * (ffcz_huffman_plan needs nalpha = 0); 0 if nalpha exceeds 2^24. */
size_t ffcz_huffman_workspace_bytes(int64_t nsym, int64_t nalpha);

/* The alphabet of a device stream of nsym symbols (min and max on the device)
 * and the sizes the encoder needs.  Blocks until they are known. */
int32_t ffcz_huffman_plan(const void* sym, int64_t nsym, int32_t width, void* workspace, size_t workspace_bytes,
                          void* stream, ffcz_huffman_sizes* plan);

/* Encode the stream into out (device, out_bytes >= the stream's size; the
 * plan's out_bytes always suffices); *used_bytes receives the size written.
 * Blocks for the frequency table (the code is built on the host) and the bit
 * count. */
int32_t ffcz_huffman_encode(const void* sym, int64_t nsym, int32_t width, const ffcz_huffman_sizes* plan,
                            void* out, size_t out_bytes, void* workspace, size_t workspace_bytes, void* stream,
                            size_t* used_bytes);

/* Decode a stream written by ffcz_huffman_encode into sym_out (device,
 * capacity symbols of the given width); *nsym_out receives the count.
 * FFCZ_E_INVALID for a corrupt header or a bit pattern that is no code. */
int32_t ffcz_huffman_decode(const void* in, size_t in_bytes, int32_t width, void* sym_out, int64_t capacity,
                            void* workspace, size_t workspace_bytes, void* stream, int64_t* nsym_out);

/* One member of a batch: shape (ndim 1..3, unit extents squeezed), device
 * pointers as in ffcz_correct, and its own bounds. */
typedef struct {
  int32_t ndim;
  int32_t pad;
  int64_t shape[3];
  const void* x_orig;
  const void* x_base;
  void* x_out;
  double eps_s;
  double delta_f;
} ffcz_instance;

/* Workspace bytes for ffcz_correct_batched over these instances (0 if one is unsupported). */
size_t ffcz_batched_workspace_bytes(int32_t dtype, int32_t count, const ffcz_instance* inst, int32_t max_iter);

/* Alg. 1 on many fields of uneven size in one call (the paper treats 1D, 2D
 * and 3D data alike, Sec. IV-C).  Members of the same 2D shape share every
 * launch (their spectra are stacked; each keeps its own bounds, counts and
 * done-flag); 3D members run one after another.  1D members take any length
 * 1..2^19, with a length-L DFT by four-step FFTs and, for lengths that are not
 * powers of two, Bluestein's chirp-z convolution.  A 1D length class runs
 * either one block per signal with the whole loop inside one launch (its work
 * buffer in LDS when it fits, see resident_1d), beside everything else, or as
 * tiled passes (many blocks per signal); tiled_1d_lg describes the choice.
 * The rounds of the grouped members and of the tiled 1D classes are enqueued
 * in chunks, each chunk one hipGraph replay (both kinds as parallel branches
 * of one graph when the batch has both), with one host poll of the done-flags
 * per chunk; the call returns when every member is finished and verified.
 * The first call with a new shape or length class may time tile variants and
 * the 1D forms on the call's own data (see ffcz_set_tuning).  Options as in
 * ffcz_correct except that masks and per-round counts are not recorded.
 * stats: NULL or a host array[count].  Returns the worst member status
 * (negative if any member failed). */
int32_t ffcz_correct_batched(int32_t dtype, int32_t count, const ffcz_instance* inst, int32_t max_iter,
                             const ffcz_options* opts, void* workspace, size_t workspace_bytes, void* stream,
                             ffcz_stats* stats);

/* Vector-Jacobian product of the fixed-round map x_hat -> y (fixed_iterations
 * = 1, `rounds` blocks) recorded by ffcz_correct into `masks`.  With the clips
 * frozen, block k is eps -> M_s^k (F^-1 M_f^k F eps); F^-1 M_f^k F is
 * symmetric (orthogonal cos/sin basis, Sec. IV-A), so
 *   grad_base = M_s^0 (A_1 (M_s^1 ... A_K (M_s^K grad_out))),  A_k = F^-1 M_f^k F.
 * The FP32 output clamp is taken as the identity.  dL/dx = grad_out - grad_base.
 *   masks     device buffer written by ffcz_correct (same shape, rounds)
 *   grad_out  dL/dy (device, dtype)       grad_base  dL/dx_hat (device, dtype)
 * Asynchronous (no host synchronisation). */
int32_t ffcz_correct_backward(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t rounds,
                              const void* masks, const void* grad_out, void* grad_base,
                              void* workspace, size_t workspace_bytes, void* stream);

/* Per-pass device timing for benchmarking.  While enabled, every launch made
 * by ffcz_correct / ffcz_correct_backward on this host thread is bracketed by
 * HIP events on the call's stream; launches that returned at entry because the
 * loop had already finished are not counted.  Pass kinds (index into ms/count):
 *   0 init (eps0, guard clip, R2C)   1 y-forward   2 x-pass (forward, count,
 *   clip, inverse)   3 y-inverse   4 z-pass (C2R, clip, R2C)   5 finalize
 *   6-8 FP64 verification z / y / x   9-11 adjoint z / y / x.
 * ffcz_profile_enable(1) also resets the sums; ffcz_profile_read waits for the
 * recorded events, returns the sums and resets them. */
#define FFCZ_PROFILE_KINDS 12
typedef struct {
  double ms[FFCZ_PROFILE_KINDS];
  int64_t count[FFCZ_PROFILE_KINDS];
} ffcz_profile;
void ffcz_profile_enable(int32_t on);
int32_t ffcz_profile_read(ffcz_profile* out);
/* Time only the pass kinds whose bit (1 << kind index above) is set in kinds; the
 * other launches run without events, so the timed passes' neighbours are not
 * slowed by event records.  0 (the default) times every kind.  Applies to calls
 * made on this host thread while profiling is enabled; ffcz_profile_enable does
 * not change it. */
void ffcz_profile_select(uint32_t kinds);

/* Plan tuning of the loop passes.  Each pass (y-forward/inverse, x-pass,
 * last-axis pass) can run with a few tilings (columns or rows per block) that
 * give bit-identical results and differ only in speed; the last-axis passes
 * also have a radix-8 stage plan (the default is radix 16) and, for FP32 rows of
 * 256 entries, a direct form (rows moved straight between HBM and registers),
 * both of which round differently.
 *   mode 0  always the default plans;
 *   mode 1  (default) on the first use of a pass geometry on a device
 *           architecture, time every variant once on the call's own workspace
 *           (a few launches, before the correction starts; skipped while the
 *           stream is being captured or masks are recorded) and keep the
 *           fastest for the rest of the process;
 *   mode 2  always the narrower tilings (for testing);
 *   mode 3  always the radix-8 last-axis plan (for testing);
 *   mode 4  always the direct last-axis loop pass (FP32 rows of 256 entries,
 *           lanes index-fastest; elsewhere the narrower tiling; for testing).
 * cache_path: JSON file of decisions, read now and rewritten after each new
 * decision; NULL keeps the current path, "" stops persisting.  The initial
 * mode and path come from FFCZ_AUTOTUNE (0 selects mode 0) and
 * FFCZ_PLAN_CACHE.  Returns FFCZ_E_INVALID for an unknown mode. */
int32_t ffcz_set_tuning(int32_t mode, const char* cache_path);
/* Forget every decision held in memory (the cache file is left as it is). */
void ffcz_clear_tuning(void);

/* Device-to-device streaming copy of `bytes` bytes: one 16-byte load and
 * store per lane, one 256-lane block per 4 KiB (the fastest simple copy
 * measured on MI355X).  A measurement helper: its rate is the HBM ceiling
 * the passes are compared with, and its read/write byte counters calibrate
 * those of the passes.  src and dst are device pointers, 16-byte aligned, not
 * overlapping; the caller owns both.  Asynchronous on `stream`.  Returns
 * FFCZ_E_INVALID for null or misaligned pointers, FFCZ_E_HIP if the launch
 * fails. */
int32_t ffcz_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Strided copy with the access pattern of the strided-axis passes (x- and
 * y-direction), the ceiling those passes are compared with.  For every
 * f < n_fixed and i < n_axis it copies row_bytes bytes at byte offset
 * f * fixed_stride + i * axis_stride from src to dst; one 256-lane block per
 * (f, 128-byte tile of the row) walks i, 16 bytes per lane.  The x-pass
 * pattern of a 3D spectrum is axis = x-planes (axis_stride = plane bytes),
 * fixed = rows (fixed_stride = row pitch); the y-pass pattern swaps them.  A
 * measurement helper, like ffcz_copy.  src and dst are device pointers the
 * caller owns, not overlapping, each holding (n_fixed - 1) * fixed_stride +
 * (n_axis - 1) * axis_stride + row_bytes bytes; the rows must not overlap one
 * another.  Asynchronous on `stream`.  Returns FFCZ_E_INVALID for negative
 * arguments, null pointers, pointers, strides or row_bytes that are not
 * multiples of 16 bytes, or more than 2^31 - 1 blocks; FFCZ_E_HIP if the
 * launch fails.  Zero counts or row_bytes copy nothing. */
int32_t ffcz_copy_columns(void* dst, const void* src, int64_t n_axis, int64_t axis_stride, int64_t n_fixed,
                          int64_t fixed_stride, int64_t row_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FFCZ_H */
