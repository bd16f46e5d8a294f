// C ABI and host driver of the correction (declarations and contracts in ffcz.h).
//
// Per projection round the device runs, for a 3D field n0 x n1 x n2 with
// half-spectrum rows of H+1 = n2/2+1 entries:
//   y-fwd   Z -> A   C2C along axis 1
//   x-pass  A -> A   C2C along axis 0, count violations, clip Re/Im, inverse C2C
//   ctl     one block per instance: sum the counts, decide on the device
//   y-inv   A -> A   inverse C2C along axis 1
//   z-pass  A -> Z   C2R along axis 2, 1/N, clip eps, R2C
// (2D: x-pass Z -> A, ctl, z-pass A -> Z; 1D fields: the x-pass has length 1.)
// Z therefore always holds the last-axis R2C of the iterate whose check is
// running, so when that check passes the output is the C2R of Z.  Every loop
// kernel returns at entry once its instance's done-flag is set, so the host
// enqueues rounds in chunks and polls the flags once per chunk.
//
// A plan covers B instances of one shape (B = 1 for ffcz_correct): their
// spectra are stacked, so one launch of each pass serves all of them, while
// every instance keeps its own bounds, counts and done-flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ffcz.h"
#include "common.hpp"
#include "kernels_bounds.hpp"
#include "kernels_edit.hpp"
#include "kernels_huff.hpp"
#include "kernels_sig.hpp"
#include "launch.hpp"
#include "sig_dispatch.hpp"

namespace ffcz {
hipError_t launch_col_f32(int mode, int L, int v, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_col_f64(int mode, int L, int v, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_row_f32(int mode, int H, int v, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_row_f64(int mode, int H, int v, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_row_f64_f32io(int mode, int H, int v, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_sig_f32(int mode, int lgMc, const void* args, int nb, hipStream_t s);
hipError_t launch_sig_f64(int mode, int lgMc, const void* args, int nb, hipStream_t s);
hipError_t launch_sigt_f64(int mode, int iodt, int lgMc, const void* args, int nb, hipStream_t s);
hipError_t launch_edit_row_f32(int mode, int H, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_edit_row_f64(int mode, int H, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_edit_col_f32(int mode, int L, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_edit_col_f64(int mode, int L, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_bounds_row_f32(int mode, int H, int vv, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_bounds_row_f64(int mode, int H, int vv, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_bounds_col_f32(int mode, int L, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_bounds_col_f64(int mode, int L, const void* args, int64_t nb, hipStream_t s);

// Which instantiation family runs a mode: the loop in the data type, set-up and
// verification in FP64 (SigArgs<double>).
bool sig_mode_fp64(int mode, int iodt) {
  const bool loop = mode == SIG_RUN || mode == SIG_RUNL || mode == SIGT_EPS0 || mode == SIGT_CIN || mode == SIGT_RMUL ||
                    mode == SIGT_RMULI ||
                    mode == SIGT_RCHECK || mode == SIGT_CCHECK || mode == SIGT_CSPAT || mode == SIGT_Y;
  return !loop || iodt == 1;
}

// iodt: data type of the batch; nsig: signals of the length class (the launch covers their tiles)
hipError_t launch_sig(int iodt, int mode, int lgMc, const void* args, int nsig, hipStream_t s) {
  const bool verify_t = mode == SIGT_VCOL || mode == SIGT_VROW || mode == SIGT_VCOL2;
  const bool setup = mode == SIG_SETUP || mode == SIGT_CHIRP || mode == SIGT_BCOL || mode == SIGT_BROW;
  if (iodt == 0) {
    if (verify_t) return launch_sigt_f64(mode, 0, lgMc, args, nsig, s);
    if (setup) return launch_sig_f64(mode, lgMc, args, nsig, s);
    return launch_sig_f32(mode, lgMc, args, nsig, s);
  }
  if (sig_tiled(mode) && !setup) return launch_sigt_f64(mode, 1, lgMc, args, nsig, s);
  return launch_sig_f64(mode, lgMc, args, nsig, s);
}

// Rows per row tile of the per-signal kernel (mirror of SigGeom).
int sig_rows_per_tile(int tdt, int lgMc) {
  const int MA = 1 << ((lgMc + 1) / 2), MB = (1 << lgMc) / MA;
  const int PA = MA / pick_E(MA), PB = MB / pick_E(MB);
  const int NT = imin3(512, MA * PB, MB * PA);
  (void)tdt;
  return NT / PA;
}

int col_block_cols(int dtype, int L, int v) { return dtype == 0 ? tile_cols<float>(L, v) : tile_cols<double>(L, v); }
int row_block_rows(int dtype, int H, int v) { return dtype == 0 ? tile_rows<float>(H, v) : tile_rows<double>(H, v); }

hipError_t launch_col(int dtype, int mode, int L, int v, const void* args, int64_t nb, hipStream_t s) {
  if (mode == COL_XEDIT || mode == COL_XUNDO)  // edit bookkeeping: default tiles only
    return dtype == 0 ? launch_edit_col_f32(mode, L, args, nb, s) : launch_edit_col_f64(mode, L, args, nb, s);
  if (mode == COL_XPASSP || mode == COL_VERIFYP)  // pointwise bounds: default tiles only
    return dtype == 0 ? launch_bounds_col_f32(mode, L, args, nb, s) : launch_bounds_col_f64(mode, L, args, nb, s);
  return dtype == 0 ? launch_col_f32(mode, L, v, args, nb, s) : launch_col_f64(mode, L, v, args, nb, s);
}
}  // namespace ffcz

using namespace ffcz;

// Scratch of ffcz_correct_noalloc: a fixed device array, one copy per GPU, held until the
// process ends.
constexpr size_t kScratchBytes = (size_t)FFCZ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(FFCZ_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// ---------------------------------------------------------------------------
// Optional per-pass timing: HIP events recorded on the call's stream around
// every launch.  Launches that return at entry because the loop already
// finished are dropped once the call knows its round count.
enum ProfKind {
  PK_INIT = 0, PK_YFWD, PK_XPASS, PK_YINV, PK_ZPASS, PK_FINAL, PK_VZ, PK_VY, PK_VX, PK_BZ, PK_BY, PK_BX,
  PK_COUNT
};
struct ProfEv {
  hipEvent_t a, b;
  int kind, round;
  int keep;  // -1: undecided (loop launch), 0: drop, 1: keep
};
struct Profiler {
  bool on = false;
  uint32_t kinds = 0;  // kinds timed (bit per kind); 0: every kind
  std::vector<ProfEv> pending;
  std::vector<hipEvent_t> pool;
  double ms[PK_COUNT] = {0};
  int64_t cnt[PK_COUNT] = {0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
thread_local Profiler g_prof;

// Wrap one launch.  round < 0 marks launches that always do work.
template <typename F>
hipError_t timed(int kind, int round, hipStream_t s, F&& launch) {
  if (!g_prof.on || (g_prof.kinds != 0 && !((g_prof.kinds >> kind) & 1u))) return launch();
  ProfEv ev{g_prof.get(), g_prof.get(), kind, round, round < 0 ? 1 : -1};
  if (ev.a) (void)hipEventRecord(ev.a, s);
  hipError_t e = launch();
  if (ev.b) (void)hipEventRecord(ev.b, s);
  if (ev.a && ev.b) g_prof.pending.push_back(ev);
  return e;
}

// Decide which loop launches of the finished call did work.
void prof_settle(int rounds) {
  for (auto& ev : g_prof.pending) {
    if (ev.keep != -1) continue;
    if (ev.kind == PK_YFWD || ev.kind == PK_XPASS) ev.keep = ev.round <= rounds;
    else ev.keep = ev.round < rounds;
  }
}

constexpr int kMaxLast = 4096;  // last axis (H <= 2048)

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// squeeze unit extents
int squeeze(int32_t ndim, const int64_t* shape, int64_t* sq) {
  int nd = 0;
  for (int i = 0; i < ndim; ++i)
    if (shape[i] > 1) sq[nd++] = shape[i];
  return nd;
}

// Fields the multidimensional plan does not take -- after squeezing, a single point or
// one axis whose length is not a power of two in [2, 4096] -- run on the 1D signal path
// (four-step or Bluestein DFT of any length up to 2^19) as a batch of one.
bool route_1d(int32_t ndim, const int64_t* shape) {
  if (ndim < 1 || ndim > 3 || !shape) return false;
  for (int i = 0; i < ndim; ++i)
    if (shape[i] < 1) return false;
  int64_t sq[3];
  const int nd = squeeze(ndim, shape, sq);
  if (nd == 0) return true;
  return nd == 1 && !(is_pow2(sq[0]) && sq[0] >= 2 && sq[0] <= kMaxLast);
}

ffcz_instance one_instance(int32_t ndim, const int64_t* shape, const void* x, const void* xb, void* y, double E,
                           double D) {
  ffcz_instance in;
  memset(&in, 0, sizeof(in));
  in.ndim = ndim;
  for (int i = 0; i < 3; ++i) in.shape[i] = i < ndim ? shape[i] : 1;
  in.x_orig = x;
  in.x_base = xb;
  in.x_out = y;
  in.eps_s = E;
  in.delta_f = D;
  return in;
}

// Partial-sum slots of the on-device margin reduction of one field: a field of
// n points uses ulp_slots(n) of them (about 16 Ki points per slot), the same
// in a single call and in a batch, so both derive the same mu.
constexpr int kUlpSlots = 1024;
__host__ __device__ inline int ulp_slots(int64_t n) {
  const int64_t k = (n + 16383) / 16384;
  return (int)(k < 1 ? 1 : (k > kUlpSlots ? kUlpSlots : k));
}

struct Plan {
  int dt = 0;        // 0 f32, 1 f64
  int nd = 0;        // squeezed ndim
  int64_t B = 1;     // instances of this shape
  int64_t n[3] = {1, 1, 1};
  int64_t N = 1;     // points per instance
  int H = 0;         // n_last / 2
  int64_t ncols = 0; // H + 1
  int64_t pitch = 0; // complex entries per spectrum row (working type)
  int64_t pitch64 = 0;
  // complex entries per x-plane (3D: n1 rows plus one 128-byte line, so that the x-direction
  // passes do not stride by a round multiple of the memory interleave; else a whole instance)
  int64_t plane = 0, plane64 = 0;
  int lg_rpp = 0;    // log2 of the spectrum rows per plane
  int64_t nrows = 0; // spectrum rows per instance
  int Lx = 1, Ly = 0;
  int Ez = 1, Ey = 1, Ex = 1;
  int64_t twz = 0, twy = 0, twx = 0, twz8 = 0, twT = 0;  // twz8: last-axis tables of the radix-8 plan
  int Ez8 = 1;
  // tile variants of the loop passes (y-forward/inverse, x-pass, last-axis init/loop/final)
  int vy = 0, vx = 0, vz = 0;
  // blocks of each pass per instance (one partial slot per block)
  int64_t zbpi = 0, ibpi = 0, vzbpi = 0, xbpi = 0, vxbpi = 0;  // ibpi: the init pass (default tiles)
  int64_t pmax = 0;
  size_t off_state = 0, off_ulp = 0, off_viol = 0, off_init = 0, off_part = 0, off_twT = 0, off_tw64 = 0, off_Z = 0,
         off_A = 0, off_W = 0, bytes = 0;
  int32_t max_iter = 0;
  int64_t s_row_w32 = 0, s_plane_bytes = 0, f_row_bytes = 0, f_plane_bytes = 0;
};

struct StateInit {
  double E, Ep, Delta, Dc, Dp, inv_n, mu, mu_s;
  int32_t max_iter, fixed, record_masks, pad;
  const void* px;
  const void* pxb;
  void* py;
  const void* pE;
  const void* pD;
  int32_t disk, pad2;
};

// Check threshold and projection bound of the f-cube.  An FP64 output is
// checked against Delta and projected onto Delta (1 - mu) (Sec. IV-B).  An FP32
// output moves every spectral component by up to mu Delta when it is rounded,
// and a coefficient accepted just below the check is never clipped, so the
// check runs mu Delta below Delta and the projection mu Delta below the check.
__host__ __device__ void spectral_thresholds(int dt, double delta, double mu, double* dc, double* dp) {
  const double rho = dt == FFCZ_F64 ? 0.0 : mu;
  *dc = delta * (1.0 - rho);
  *dp = delta * (1.0 - rho - mu);
}

int ceil_lg(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

// The FP64 last-axis verification pass runs the radix-8 plan: half the registers
// per lane of radix 16, so twice the lanes of an FP64 row tile stay resident.
constexpr int kVerifyRowPlan = 2;

// FP64 fields: the closing pass runs on the radix-8 tiles of the verification and, when
// verification is on, goes on to the verification's last-axis R2C in the same pass (x and
// y read once): rows of up to 512 entries, where those tiles still hold 4 or more rows.  The
// closing pass takes the same form with verification off, so y does not depend on it.  (For
// FP32 fields the fused pass would move the closing C2R into FP64 arithmetic, and measured
// slower than the two passes.)
bool final_fused(const Plan& p) { return p.dt == FFCZ_F64 && p.H >= 2 && p.H <= 512; }

// Choose the loop passes' tile variants and the per-instance block counts that follow.
// Plan of the init, closing and adjoint last-axis passes: the direct form (variant 3)
// when the loop pass runs it on 128- or 256-entry FP32 rows, else the default tiles
// (the closing pass of FP64 fields with rows of up to 512 entries: see final_fused).
int init_variant(const Plan& p) {
  return (p.vz == 3 && p.dt == FFCZ_F32 && (p.H == 128 || p.H == 256)) ? 3 : 0;
}

// Neighbouring column tiles that read parts of the same 128-byte lines (1 when a tile row fills
// a line), and the tiles per outer index, padded to a multiple of that so that each group of
// neighbours runs on one XCD (xcd_tile; padding tiles hold no column).  FFCZ_XCD_ORDER=0 keeps
// the plain order (for measurement); both orders give identical bits.
bool xcd_order_on() {
  static const bool on = [] {
    const char* e = getenv("FFCZ_XCD_ORDER");
    return !(e && e[0] == '0');
  }();
  return on;
}
int col_line_share(int dt, int L, int v) {
  const int row_bytes = col_block_cols(dt, L, v) * (dt == FFCZ_F32 ? 8 : 16);
  return (xcd_order_on() && row_bytes < 128) ? 128 / row_bytes : 1;
}
int64_t col_tiles(int dt, int L, int v, int64_t ncols) {
  const int C = col_block_cols(dt, L, v), k = col_line_share(dt, L, v);
  return ((ncols + C - 1) / C + k - 1) / k * k;
}

void set_variants(Plan& p, int vy, int vx, int vz) {
  p.vy = vy;
  p.vx = vx;
  p.vz = vz;
  const int64_t outer_x = p.nd == 3 ? p.n[1] : 1;
  const int Rz = row_block_rows(p.dt, p.H, vz), Rz64 = row_block_rows(1, p.H, kVerifyRowPlan);
  p.zbpi = (p.nrows + Rz - 1) / Rz;
  const int Ri = row_block_rows(p.dt, p.H, init_variant(p));
  p.ibpi = (p.nrows + Ri - 1) / Ri;
  p.vzbpi = (p.nrows + Rz64 - 1) / Rz64;
  p.xbpi = outer_x * col_tiles(p.dt, p.Lx, vx, p.ncols);
  p.vxbpi = outer_x * col_tiles(FFCZ_F64, p.Lx, 0, p.ncols);
}

int32_t make_plan(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter, int64_t B, Plan& p) {
  if (dtype != FFCZ_F32 && dtype != FFCZ_F64) return fail(FFCZ_E_INVALID, "dtype must be FFCZ_F32 or FFCZ_F64");
  if (ndim < 1 || ndim > 3 || shape == nullptr) return fail(FFCZ_E_SHAPE, "ndim must be 1..3");
  if (max_iter < 0) return fail(FFCZ_E_INVALID, "max_iter must be >= 0");
  p = Plan();
  p.dt = dtype;
  p.max_iter = max_iter;
  p.B = B;
  for (int i = 0; i < ndim; ++i)
    if (shape[i] < 1) return fail(FFCZ_E_SHAPE, "every extent must be >= 1");
  int64_t sq[3];
  const int nd = squeeze(ndim, shape, sq);
  if (nd == 0) return fail(FFCZ_E_SHAPE, "a single-point field is not supported (last extent must be >= 2)");
  const int64_t maxo = dtype == FFCZ_F32 ? 2048 : 1024;
  for (int i = 0; i < nd; ++i) {
    if (!is_pow2(sq[i])) return fail(FFCZ_E_SHAPE, "extents must be powers of two");
    if (i < nd - 1 && sq[i] > maxo) return fail(FFCZ_E_SHAPE, "leading extents above the supported maximum");
  }
  const int64_t nl = sq[nd - 1];
  if (nl < 2 || nl > kMaxLast) return fail(FFCZ_E_SHAPE, "last extent must be in [2, 4096]");
  if (nd == 3 && B != 1) return fail(FFCZ_E_SHAPE, "3D instances are corrected one at a time");
  p.nd = nd;
  for (int i = 0; i < nd; ++i) p.n[i] = sq[i];
  p.N = 1;
  for (int i = 0; i < nd; ++i) p.N *= sq[i];
  p.H = (int)(nl / 2);
  p.ncols = p.H + 1;
  const int64_t cT = dtype == FFCZ_F32 ? 16 : 8;  // 128-byte pitch alignment
  p.pitch = align_up(p.ncols, cT);
  p.pitch64 = align_up(p.ncols, 8);
  p.nrows = p.N / nl;
  p.Lx = nd >= 2 ? (int)sq[0] : 1;
  p.Ly = nd == 3 ? (int)sq[1] : 0;
  p.Ez = pick_E_row(p.H);
  p.Ex = pick_E(p.Lx);
  p.Ey = p.Ly ? pick_E(p.Ly) : 1;
  p.twz = 0;
  p.twy = p.twz + host_twsize(p.H, p.Ez) + p.H;
  p.twx = p.twy + (p.Ly ? host_twsize(p.Ly, p.Ey) : 0);
  p.Ez8 = row_E(p.H, 2);
  p.twz8 = p.twx + host_twsize(p.Lx, p.Ex) + 1;
  p.twT = p.twz8 + host_twsize(p.H, p.Ez8) + p.H;
  const size_t cs = dtype == FFCZ_F32 ? 8 : 16;
  set_variants(p, 0, 0, 0);
  {
    // partial slots for the narrowest tiles any variant uses
    const int64_t outer_x = nd == 3 ? p.n[1] : 1;
    int64_t xtiles = 0;
    for (int v = 0; v < kColVariants; ++v) xtiles = std::max(xtiles, col_tiles(dtype, p.Lx, v, p.ncols));
    int Rmin = row_block_rows(dtype, p.H, 0);
    for (int v = 1; v < kRowVariants; ++v) Rmin = std::min(Rmin, row_block_rows(dtype, p.H, v));
    const int64_t zmax = (p.nrows + Rmin - 1) / Rmin, xmax = outer_x * xtiles;
    p.pmax = B * std::max(std::max(zmax, p.vzbpi), std::max(xmax, p.vxbpi));
  }
  size_t off = 0;
  p.off_state = off;
  off = align_up(off + sizeof(DevState) * (size_t)B, 256);
  p.off_ulp = off;  // margin reduction: kUlpSlots partial sums, then mu
  off = align_up(off + sizeof(double) * (kUlpSlots + 1), 256);
  p.off_viol = off;
  off = align_up(off + sizeof(unsigned long long) * ((size_t)max_iter + 2) * (size_t)B, 256);
  p.off_init = off;
  off = align_up(off + (B > 1 ? sizeof(StateInit) * (size_t)B : 0), 256);
  // partial slots: x-pass counts | z-pass counts | verify-z max | verify-x count, max
  p.off_part = off;
  off = align_up(off + sizeof(unsigned long long) * 5 * (size_t)p.pmax, 256);
  p.off_twT = off;
  off = align_up(off + cs * (size_t)p.twT, 256);
  p.off_tw64 = off;
  off = align_up(off + 16 * (size_t)p.twT, 256);
  p.off_Z = off;
  const int64_t rpp = nd == 3 ? p.n[1] : p.nrows;
  p.lg_rpp = ceil_lg(rpp);
  p.plane = rpp * p.pitch + (nd == 3 ? cT : 0);
  p.plane64 = rpp * p.pitch64 + (nd == 3 ? 8 : 0);
  const size_t nplanes = (size_t)B * (size_t)(p.nrows / rpp);
  const size_t spec = cs * nplanes * (size_t)p.plane;
  off = align_up(off + spec, 256);
  p.off_A = off;
  off = align_up(off + spec, 256);
  // the FP64 verification spectrum reuses Z..A (contiguous) once y is written; the fused
  // closing pass reads Z while it writes, so there it starts at A (free once the loop ends)
  p.off_W = final_fused(p) ? p.off_A : p.off_Z;
  const size_t spec64 = 16 * nplanes * (size_t)p.plane64;
  if (p.off_W + spec64 > off) off = align_up(p.off_W + spec64, 256);
  p.bytes = off;
  const int64_t sw64 = (nl + 63) / 64;
  const int64_t fw64 = (p.ncols + 63) / 64;
  p.s_row_w32 = 2 * sw64;
  p.s_plane_bytes = p.nrows * sw64 * 8;
  p.f_row_bytes = fw64 * 8;
  p.f_plane_bytes = p.nrows * fw64 * 8;
  return FFCZ_OK;
}

// ---------------------------------------------------------------------------
// set-up, control and statistics kernels

struct TwJob {
  int64_t off;  // complex entries from the table base
  int L, E, rtw;
};
struct TwJobs {
  TwJob j[4];
  int n;
  int dbl;  // 1: double table
};

// Stage twiddles exp(-2 pi i m r / (Ns R)) and R2C twiddles exp(-2 pi i k / 2L),
// evaluated in FP64 with an exactly reduced argument and rounded once.
// blockIdx.y picks one of two tables (base0/jobs0 or base1/jobs1), so a plan's
// working-precision and FP64 tables take one launch.
__global__ void twiddle_kernel(void* base0, TwJobs jobs0, void* base1, TwJobs jobs1) {
  void* const base = blockIdx.y ? base1 : base0;
  const TwJobs& jobs = blockIdx.y ? jobs1 : jobs0;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t acc = 0;
  for (int jj = 0; jj < jobs.n; ++jj) {
    const TwJob& jb = jobs.j[jj];
    // the stage plan of host_twsize, walked without a table (no per-lane scratch)
    const int64_t tsz = jb.E > 1 && jb.L > 1 ? host_twsize(jb.L, jb.E) : 0;
    const int64_t cnt = tsz + (jb.rtw ? jb.L : 0);
    if (gid < acc + cnt) {
      const int64_t e = gid - acc;
      double num, den;  // angle = -2 pi num / den
      if (e < tsz) {
        const int lgE = ilog2c(jb.E), a = ilog2c(jb.L) / lgE;
        const int r0 = jb.L >> (a * lgE);
        int64_t ns = r0 > 1 ? r0 : 1, off = 0;
        for (int t = 0; t < a; ++t, ns *= jb.E) {
          if (ns == 1) continue;
          const int64_t own = ns * (jb.E - 1);
          if (e < off + own) break;
          off += own;
        }
        const int64_t loc = e - off;
        const int64_t m = loc / (jb.E - 1);
        const int64_t r = loc % (jb.E - 1) + 1;
        num = (double)(m * r);
        den = (double)ns * jb.E;
      } else {
        num = (double)(e - tsz);
        den = 2.0 * jb.L;
      }
      double sn, cs;
      sincospi(-2.0 * num / den, &sn, &cs);
      if (jobs.dbl) {
        cx<double>* t = (cx<double>*)base + jb.off + e;
        *t = cx<double>{cs, sn};
      } else {
        cx<float>* t = (cx<float>*)base + jb.off + e;
        *t = cx<float>{__double2float_rn(cs), __double2float_rn(sn)};
      }
      return;
    }
    acc += cnt;
  }
}

__global__ void state_init_kernel(DevState* st, int64_t B, const StateInit* arr, StateInit one,
                                  unsigned long long* viol, int64_t nviol) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < B) {
    const StateInit p = arr ? arr[t] : one;
    DevState s;
    memset(&s, 0, sizeof(s));
    s.E = p.E;
    s.Ep = p.Ep;
    s.Delta = p.Delta;
    s.Dc = p.Dc;
    s.Dp = p.Dp;
    s.inv_n = p.inv_n;
    s.mu = p.mu;
    s.mu_s = p.mu_s;
    s.max_iter = p.max_iter;
    s.fixed = p.fixed;
    s.record_masks = p.record_masks;
    s.px = p.px;
    s.pxb = p.pxb;
    s.py = p.py;
    s.pE = p.pE;
    s.pD = p.pD;
    s.disk = p.disk;
    s.fe = 1.0 - p.mu;
    s.fc = 1.0;
    s.fp = 1.0 - p.mu;
    st[t] = s;
  }
  for (int64_t i = t; i < nviol; i += (int64_t)gridDim.x * blockDim.x) viol[i] = 0ull;
}

// Suggested FP32 margin for a field of N points with bound Delta:
// mu = max(2^-16, 8 sigma sqrt(N/2) / Delta), sigma^2 = mean(ulp(x)^2) / 12, at
// most 1/2.  Rounding y to FP32 moves each Re/Im component of its spectrum by
// sigma sqrt(N/2) rms (N independent roundings of variance ulp^2/12, half of
// each in the real part).  A non-finite sum gives 2^-16 (NaN) or 1/2 (Inf);
// such inputs stop the correction anyway.
__host__ __device__ double margin_from_ulp2(double ulp2_sum, int64_t N, double D) {
  const double sigma = sqrt(ulp2_sum / (double)N / 12.0);
  const double m = D > 0 ? 8.0 * sigma * sqrt((double)N / 2.0) / D : 0.5;
  const double lo = 0x1p-16;
  const double a = lo < m ? m : lo;
  return a < 0.5 ? a : 0.5;
}

// One field of a margin computation: x (FP32, N points) and its bound Delta.
struct MarginJob {
  const float* x;
  int64_t n;
  double D;
};

// ulp(v)^2 = (nextafter(|v|, +Inf) - |v|)^2 from the exponent field e of v:
// 2^(2 max(e, 1) - 300), exact in FP64; FLT_MAX steps to Inf, Inf and NaN give NaN.
__device__ inline double ulp2f(float v) {
  const uint32_t b = __float_as_uint(v) & 0x7fffffffu;
  const uint32_t e = b >> 23;
  if (e == 255u) return __longlong_as_double(0x7ff8000000000000ll);
  if (b == 0x7f7fffffu) return __longlong_as_double(0x7ff0000000000000ll);
  const int64_t ex = 2 * (int64_t)(e > 0u ? e : 1u) - 300 + 1023;
  return __longlong_as_double(ex << 52);
}

// Partial sums of ulp(x)^2.  blockIdx.y picks the field (jobs[y], or `one`
// when jobs is null); its points are cut into nb = ulp_slots(n) contiguous
// slices of a multiple of 4 points, and block b < nb stores the sum over slice
// b in part[y * kUlpSlots + b] (blocks past nb have nothing to do).  No
// atomics: margin_kernel adds the slots in a fixed order, so mu does not
// depend on scheduling.  Aligned slices stream 16-byte vectors, four in flight
// per lane.
__global__ void __launch_bounds__(256) ulp_part_kernel(MarginJob one, const MarginJob* jobs, double* part) {
  __shared__ double red[4];
  const MarginJob jb = jobs ? jobs[blockIdx.y] : one;
  const int64_t nb = ulp_slots(jb.n);
  if ((int64_t)blockIdx.x >= nb) return;
  const int64_t slice = ((jb.n + nb - 1) / nb + 3) & ~int64_t(3);
  const int64_t lo = std::min<int64_t>(jb.n, (int64_t)blockIdx.x * slice);
  const int64_t hi = std::min<int64_t>(jb.n, lo + slice);
  const float* x = jb.x;
  double s = 0.0;
  int64_t i0 = lo;
  if (((uintptr_t)(x + lo) & 15) == 0) {
    const float4* x4 = (const float4*)(x + lo);
    const int64_t n4 = (hi - lo) >> 2;
    constexpr int U = 4;
    int64_t k = threadIdx.x;
    for (; k + (U - 1) * 256 < n4; k += U * 256) {
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = x4[k + u * 256];
#pragma unroll
      for (int u = 0; u < U; ++u) s += ulp2f(v[u].x) + ulp2f(v[u].y) + ulp2f(v[u].z) + ulp2f(v[u].w);
    }
    for (; k < n4; k += 256) {
      const float4 v = x4[k];
      s += ulp2f(v.x) + ulp2f(v.y) + ulp2f(v.z) + ulp2f(v.w);
    }
    i0 = lo + 4 * n4;
  }
  for (int64_t i = i0 + threadIdx.x; i < hi; i += 256) s += ulp2f(x[i]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * kUlpSlots + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One block per field: add its ulp_slots(n) partial sums in a fixed order and
// derive mu.  mu_out[field] receives it when given; st (one state per field), when
// given, receives mu and the bounds that depend on it (E (1 - mu) and the
// spectral check and projection thresholds), the same values the host fills
// in when mu is supplied.
__global__ void __launch_bounds__(256) margin_kernel(const double* part, MarginJob one, const MarginJob* jobs, int dt,
                                                     double* mu_out, DevState* st) {
  __shared__ double red[4];
  const MarginJob jb = jobs ? jobs[blockIdx.x] : one;
  const int nslot = ulp_slots(jb.n);
  const double* pp = part + (int64_t)blockIdx.x * kUlpSlots;
  double s = 0.0;
  for (int k = threadIdx.x; k < nslot; k += 256) s += pp[k];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double mu = margin_from_ulp2((red[0] + red[1]) + (red[2] + red[3]), jb.n, jb.D);
  if (mu_out) mu_out[blockIdx.x] = mu;
  if (st) {
    DevState* t = st + blockIdx.x;
    t->mu = mu;
    t->Ep = t->E * (1.0 - mu);
    double dc, dp;
    spectral_thresholds(dt, t->Delta, mu, &dc, &dp);
    t->Dc = dc;
    t->Dp = dp;
  }
}


// max |x| partials of a field (one per slice, slices as in ulp_part_kernel), as the bits of
// a non-negative double (which order as integers).
template <typename TIO>
__global__ void __launch_bounds__(256) absmax_part_kernel(const TIO* x, int64_t n, unsigned long long* part) {
  __shared__ double red[4];
  const int64_t nb = ulp_slots(n);
  if ((int64_t)blockIdx.x >= nb) return;
  const int64_t slice = (n + nb - 1) / nb;
  const int64_t lo = std::min<int64_t>(n, (int64_t)blockIdx.x * slice);
  const int64_t hi = std::min<int64_t>(n, lo + slice);
  double m = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) m = fmax(m, fabs((double)x[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = (unsigned long long)__double_as_longlong(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

// Spacing of the dtype's grid just above v >= 0 (what an output of that size is rounded to).
__device__ inline double grid_spacing(int dt, double v) {
  if (dt == FFCZ_F32) {
    const float f = __double2float_rn(v);
    return (double)nextafterf(f, __builtin_huge_valf()) - (double)f;
  }
  return nextafter(v, __builtin_huge_val()) - v;
}

// Shrinks of the encoder, one block.  The paper shrinks both cubes by 2^-m so that the
// quantised edits still land inside (Sec. IV-B).  That counts each edit's own rounding
// only: the quantisation error of one domain also reaches the other through the
// transform, and the decoder rounds its output without a clamp (it does not know x).  So
// with q = safety 2^-m:
//   mu_f = max(q, mu_out)  (mu_out: the output-rounding margin of the plain correction,
//                           from the ulp partials for FP32 fields, 2^-16 for FP64),
//   mu_s = q + spacing(max|x| + E) / E  (a whole output ulp, twice its rounding error),
// capped at 1/4 and 1/2; the check runs at Delta (1 - mu_f), the f-projection at
// Delta (1 - 2 mu_f) and the s-projection at E (1 - mu_s).
__global__ void __launch_bounds__(256) encode_margin_kernel(const double* ulp_part, const unsigned long long* amax,
                                                            int64_t n, int dt, double q, DevState* st) {
  __shared__ double red[4];
  __shared__ unsigned long long redm[4];
  const int nslot = ulp_slots(n);
  double s = 0.0;
  unsigned long long mb = 0;
  for (int k = threadIdx.x; k < nslot; k += 256) {
    if (dt == FFCZ_F32) s += ulp_part[k];
    mb = mb > amax[k] ? mb : amax[k];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    const unsigned long long o = __shfl_xor(mb, off, 64);
    mb = mb > o ? mb : o;
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = s;
    redm[threadIdx.x >> 6] = mb;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < 4; ++w) redm[0] = redm[0] > redm[w] ? redm[0] : redm[w];
  const double xm = __longlong_as_double((long long)redm[0]);
  const double mu_out = dt == FFCZ_F32 ? margin_from_ulp2((red[0] + red[1]) + (red[2] + red[3]), n, st->Delta)
                                       : 0x1p-16;
  const double E = st->E;
  const double mu_f = fmin(fmax(mu_out, q), 0.25);
  const double mu_s = fmin(q + (E > 0.0 ? grid_spacing(dt, xm + E) / E : 0.0), 0.5);
  st->mu = mu_f;
  st->mu_s = mu_s;
  st->Ep = E * (1.0 - mu_s);
  st->Dc = st->Delta * (1.0 - mu_f);
  st->Dp = st->Delta * (1.0 - 2.0 * mu_f);
}

// Margin and threshold factors for pointwise bounds, one block.  FP64 output: mu = 2^-16 (or
// the caller's), check at D_k, project onto D_k (1 - mu) and E_n (1 - mu).  FP32 output: the
// FP32 rule of margin_kernel with Delta = the smallest spectral bound (times sqrt 2 for the
// disk, whose modulus takes the rounding noise of both parts), check at D_k (1 - mu), project
// onto D_k (1 - 2 mu).
__global__ void __launch_bounds__(256) bounds_margin_kernel(const double* ulp_part, const unsigned long long* minpart,
                                                            int nmin, int64_t n, int dt, int disk, double mu_given,
                                                            DevState* st) {
  __shared__ double red[4];
  __shared__ unsigned long long redm[4];
  const int nslot = ulp_slots(n);
  double s = 0.0;
  unsigned long long mb = ~0ull;
  if (dt == FFCZ_F32)
    for (int k = threadIdx.x; k < nslot; k += 256) s += ulp_part[k];
  for (int k = threadIdx.x; k < nmin; k += 256) mb = mb < minpart[k] ? mb : minpart[k];
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    const unsigned long long o = __shfl_xor(mb, off, 64);
    mb = mb < o ? mb : o;
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = s;
    redm[threadIdx.x >> 6] = mb;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < 4; ++w) redm[0] = redm[0] < redm[w] ? redm[0] : redm[w];
  double mu = mu_given;
  if (!(mu > 0.0)) {
    if (dt == FFCZ_F64) {
      mu = 0x1p-16;
    } else {
      const double dmin = redm[0] == ~0ull ? 0.0 : __longlong_as_double((long long)redm[0]);
      const double sigma = sqrt(((red[0] + red[1]) + (red[2] + red[3])) / (double)n / 12.0);
      double m = dmin > 0.0 ? 8.0 * sigma * sqrt((double)n / 2.0) / dmin : 0.5;
      if (disk && dmin > 0.0) m *= sqrt(2.0);
      mu = fmin(0.5, fmax(0x1p-16, m));
    }
  }
  const double rho = dt == FFCZ_F64 ? 0.0 : mu;
  st->mu = mu;
  st->fe = 1.0 - mu;
  st->fc = 1.0 - rho;
  st->fp = 1.0 - rho - mu;
  st->Ep = st->E * (1.0 - mu);
}

// Partials p[0..n) read by the nt lanes of a block, U independent loads in flight per lane
// (a plain strided loop waits for each load in turn: with thousands of partials that was
// most of a control kernel's time).  fold is a sum or a max of non-negative values.
template <int U, typename F>
__device__ __forceinline__ unsigned long long fold_strided(const unsigned long long* p, int64_t n, int t, int nt,
                                                           unsigned long long acc, F fold) {
  for (int64_t i0 = t; i0 < n; i0 += (int64_t)U * nt) {
    unsigned long long v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * nt;
      v[u] = i < n ? p[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = fold(acc, v[u]);
  }
  return acc;
}
__device__ __forceinline__ unsigned long long add_u64(unsigned long long a, unsigned long long b) { return a + b; }
__device__ __forceinline__ unsigned long long max_u64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }

// Per-round control, one block per instance: sum the x-pass partials into
// v_k, fold the spatial-clip partials of the z-pass that produced the checked
// iterate into the totals, and decide on the device whether the loop stops
// (Alg. 1: stop when no coefficient violates; also at the round cap, or on
// non-finite input).
__global__ void __launch_bounds__(1024) ctl_kernel(DevState* st0, unsigned long long* viol0, int64_t vstride,
                                                   const unsigned long long* xpart, int64_t xbpi,
                                                   const unsigned long long* zpart, int64_t zbpi,
                                                   int64_t ibpi) {
  __shared__ unsigned long long rx[16], rz[16];
  const int64_t b = blockIdx.x;
  DevState* st = st0 + b;
  if (*(volatile int32_t*)&st->done) return;
  const int t = threadIdx.x;
  // the checked iterate came from the init pass (round 0) or from a z-pass, whose tiles may differ
  const int64_t nz = st->round == 0 ? ibpi : zbpi;
  unsigned long long sx = fold_strided<8>(xpart + b * xbpi, xbpi, t, (int)blockDim.x, 0ull, add_u64);
  unsigned long long sz = fold_strided<8>(zpart + b * nz, nz, t, (int)blockDim.x, 0ull, add_u64);
  sx = wave_sum_u64(sx);
  sz = wave_sum_u64(sz);
  if ((t & 63) == 0) {
    rx[t >> 6] = sx;
    rz[t >> 6] = sz;
  }
  __syncthreads();
  if (t == 0) {
    unsigned long long vx = 0, vz = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
      vx += rx[w];
      vz += rz[w];
    }
    const int k = st->round;
    viol0[b * vstride + k] = vx;
    if (k == 0) st->v_first = vx;
    st->v_last = vx;
    if (k == 0) st->s_guard = vz;
    else st->s_clipped_total += vz;
    int stop = 0;
    if (st->nonfinite) {
      stop = 1;
      st->nonfinite_stop = 1;
    } else if (!st->fixed && vx == 0) {
      stop = 1;
      st->converged = 1;
    } else if (k >= st->max_iter) {
      stop = 1;
      st->converged = (vx == 0) ? 1 : 0;
    }
    if (stop) st->done = 1;
    else st->round = k + 1;
  }
}

// Reduce the verification partials of each instance: max |y - x|,
// max(|Re|,|Im|) and the count above Delta.
__global__ void __launch_bounds__(1024) stats_kernel(DevState* st0, const unsigned long long* vz, int64_t vzbpi,
                                                     const unsigned long long* vxc, const unsigned long long* vxm,
                                                     int64_t vxbpi) {
  __shared__ unsigned long long ra[16], rb[16], rc[16];
  const int64_t inst = blockIdx.x;
  const int t = threadIdx.x;
  // max bits of non-negative doubles order as integers
  unsigned long long a = fold_strided<8>(vz + inst * vzbpi, vzbpi, t, (int)blockDim.x, 0ull, max_u64);
  unsigned long long b = fold_strided<8>(vxm + inst * vxbpi, vxbpi, t, (int)blockDim.x, 0ull, max_u64);
  unsigned long long c = fold_strided<8>(vxc + inst * vxbpi, vxbpi, t, (int)blockDim.x, 0ull, add_u64);
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long oa = __shfl_xor(a, off, 64), ob = __shfl_xor(b, off, 64);
    a = a > oa ? a : oa;
    b = b > ob ? b : ob;
    c += __shfl_xor(c, off, 64);
  }
  if ((t & 63) == 0) {
    ra[t >> 6] = a;
    rb[t >> 6] = b;
    rc[t >> 6] = c;
  }
  __syncthreads();
  if (t == 0) {
    unsigned long long A = 0, Bm = 0, Cc = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
      A = A > ra[w] ? A : ra[w];
      Bm = Bm > rb[w] ? Bm : rb[w];
      Cc += rc[w];
    }
    st0[inst].max_spatial_bits = A;
    st0[inst].max_spectral_bits = Bm;
    st0[inst].spectral_viol = Cc;
  }
}

// ---------------------------------------------------------------------------

struct Ctx {
  const Plan* p;
  char* ws;
  hipStream_t s;
  // edit accumulators (encoder only): spatial, one value per point; frequency, laid out as Z
  void* sacc = nullptr;
  void* facc = nullptr;
  // pointwise bounds: the (Re, Im) bound pairs laid out as Z (null: the scalar bounds)
  const void* pD = nullptr;
  DevState* st() const { return (DevState*)(ws + p->off_state); }
  unsigned long long* viol() const { return (unsigned long long*)(ws + p->off_viol); }
  void* twT() const { return ws + p->off_twT; }
  void* tw64() const { return ws + p->off_tw64; }
  void* Z() const { return ws + p->off_Z; }
  void* A() const { return ws + p->off_A; }
  void* W() const { return ws + p->off_W; }
  unsigned long long* part(int i) const { return (unsigned long long*)(ws + p->off_part) + (size_t)i * p->pmax; }
  static constexpr int PX = 0, PZ = 1, PVZ = 2, PVX = 3;  // PVX spans two regions (count, max)
};

hipError_t launch_ctl(const Ctx& c, unsigned long long* viol, int64_t vstride) {
  hipLaunchKernelGGL(ctl_kernel, dim3((unsigned)c.p->B), dim3(1024), 0, c.s, c.st(), viol, vstride, c.part(Ctx::PX),
                     c.p->xbpi, c.part(Ctx::PZ), c.p->zbpi, c.p->ibpi);
  return hipGetLastError();
}

hipError_t write_twiddles(const Ctx& c) {
  const Plan& p = *c.p;
  // table 0: working precision (read by the loop kernels); table 1: FP64 (verification)
  TwJobs jobs[2];
  for (int tab = 0; tab < 2; ++tab) {
    memset(&jobs[tab], 0, sizeof(TwJobs));
    jobs[tab].dbl = (tab == 1 || p.dt == FFCZ_F64) ? 1 : 0;
    int n = 0;
    jobs[tab].j[n++] = TwJob{p.twz, p.H, p.Ez, 1};
    jobs[tab].j[n++] = TwJob{p.twz8, p.H, p.Ez8, 1};
    if (p.Ly) jobs[tab].j[n++] = TwJob{p.twy, p.Ly, p.Ey, 0};
    jobs[tab].j[n++] = TwJob{p.twx, p.Lx, p.Ex, 0};
    jobs[tab].n = n;
  }
  const int nb = (int)((p.twT + 255) / 256);
  hipLaunchKernelGGL(twiddle_kernel, dim3(nb, 2), dim3(256), 0, c.s, c.twT(), jobs[0], c.tw64(), jobs[1]);
  return hipGetLastError();
}

// Geometry of a strided-axis pass.
struct ColGeom {
  int L;
  int64_t outer, so, s;
  int64_t mrow_i, mrow_o;
  int64_t outer_per_inst;
  int64_t pitch;  // complex entries per row of the buffer (the padded row)
};

// pitch / plane: complex entries per spectrum row / per x-plane of the buffer addressed
ColGeom geom_y(const Plan& p, int64_t pitch, int64_t plane) {  // 3D only (B = 1)
  return ColGeom{p.Ly, p.n[0], plane, pitch, 0, 0, p.n[0], pitch};
}
ColGeom geom_x(const Plan& p, int64_t pitch, int64_t plane) {
  if (p.nd == 3) return ColGeom{p.Lx, p.n[1], pitch, plane, p.n[1], 1, p.n[1], pitch};
  // 2D (and 1D, Lx = 1): one outer index per instance (a whole instance is one plane)
  return ColGeom{p.Lx, p.B, plane, pitch, 1, 0, 1, pitch};
}

template <typename T>
hipError_t run_col(int dt, int mode, int v, const ColGeom& g, const Plan& p, const void* src, void* dst,
                   const void* tw, DevState* st, unsigned long long* part, uint8_t* fmask,
                   hipStream_t s, void* fedit = nullptr, const void* bnd = nullptr, int64_t bnd_so = 0,
                   int64_t bnd_s = 0, int bnd_dbl = 0) {
  ColArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.src = (const cx<T>*)src;
  a.dst = (cx<T>*)dst;
  a.so = g.so;
  a.s = g.s;
  a.ncols = (int32_t)p.ncols;
  a.ncols_pad = (int32_t)g.pitch;
  a.ncb = (int32_t)col_tiles(dt, g.L, v, p.ncols);
  a.xcd_k = col_line_share(dt, g.L, v);
  a.outer_per_inst = g.outer_per_inst;
  a.tw = (const cx<T>*)tw;
  a.st = st;
  a.part = part;
  a.part_stride = p.pmax;
  a.fmask = fmask;
  a.f_plane = p.f_plane_bytes;
  a.f_row_bytes = p.f_row_bytes;
  a.mrow_i = g.mrow_i;
  a.mrow_o = g.mrow_o;
  a.fedit = (cx<T>*)fedit;
  a.bnd = bnd;
  a.bnd_so = bnd_so;
  a.bnd_s = bnd_s;
  a.bnd_dbl = bnd_dbl;
  const int64_t nb = g.outer * a.ncb;
  return launch_col(dt, mode, g.L, v, &a, nb, s);
}

template <typename T, typename TIO>
hipError_t run_row(int tdt, int iodt, int mode, int v, const Plan& p, int64_t pitch, int64_t plane, const void* src,
                   void* dst, const void* tw, DevState* st, unsigned long long* part, uint32_t* smask,
                   hipStream_t s, int64_t spitch = -1, int64_t splane = -1, void* sedit = nullptr) {
  RowArgs<T, TIO> a;
  memset(&a, 0, sizeof(a));
  a.src = (const cx<T>*)src;
  a.dst = (cx<T>*)dst;
  a.pitch = pitch;
  a.spitch = spitch < 0 ? pitch : spitch;
  a.splane = splane < 0 ? plane : splane;
  a.rows_per_inst = p.nrows;
  const int R = row_block_rows(tdt, p.H, v);
  a.bpi = (p.nrows + R - 1) / R;
  a.tw = (const cx<T>*)tw;
  a.st = st;
  a.part = part;
  a.smask = smask;
  a.s_plane = p.s_plane_bytes / 4;
  a.s_row_w32 = (int32_t)p.s_row_w32;
  const int64_t nb = a.bpi * p.B;
  a.plane = plane;
  a.lg_rpp = p.lg_rpp;
  a.sedit = (T*)sedit;
  if (mode == ROW_INITE || mode == ROW_LOOPE || mode == ROW_DECODE)  // default tiles only
    return tdt == 0 ? launch_edit_row_f32(mode, p.H, &a, nb, s) : launch_edit_row_f64(mode, p.H, &a, nb, s);
  if (mode >= ROW_INITP && mode <= ROW_VERIFYP)  // pointwise bounds, by the field's dtype
    return iodt == 0 ? launch_bounds_row_f32(mode, p.H, v, &a, nb, s) : launch_bounds_row_f64(mode, p.H, v, &a, nb, s);
  if (tdt == 1 && iodt == 0) return launch_row_f64_f32io(mode, p.H, v, &a, nb, s);
  return tdt == 0 ? launch_row_f32(mode, p.H, v, &a, nb, s) : launch_row_f64(mode, p.H, v, &a, nb, s);
}

template <typename T>
hipError_t row_T(int mode, const Ctx& c, const void* src, void* dst, uint32_t* smask) {
  const Plan& p = *c.p;
  if (c.pD && (mode == ROW_INIT || mode == ROW_LOOP)) {
    // pointwise bounds: the staged pass on the default tiles
    return run_row<T, T>(p.dt, p.dt, mode == ROW_INIT ? ROW_INITP : ROW_LOOPP, 0, p, p.pitch, p.plane, src, dst,
                         (const char*)c.twT() + sizeof(cx<T>) * p.twz, c.st(), c.part(Ctx::PZ), smask, c.s);
  }
  if (c.sacc && (mode == ROW_INIT || mode == ROW_LOOP)) {
    // with edit bookkeeping: the staged pass on the default tiles
    return run_row<T, T>(p.dt, p.dt, mode == ROW_INIT ? ROW_INITE : ROW_LOOPE, 0, p, p.pitch, p.plane, src, dst,
                         (const char*)c.twT() + sizeof(cx<T>) * p.twz, c.st(), c.part(Ctx::PZ), smask, c.s, -1, -1,
                         c.sacc);
  }
  const int v = mode == ROW_LOOP ? p.vz : init_variant(p);
  const void* tw = (const char*)c.twT() + sizeof(cx<T>) * (v == 2 ? p.twz8 : p.twz);
  return run_row<T, T>(p.dt, p.dt, mode, v, p, p.pitch, p.plane, src, dst, tw, c.st(), c.part(Ctx::PZ), smask, c.s);
}

// The loop's x-pass: plain, with edit bookkeeping, or against pointwise bounds (the bound
// pairs share the spectrum's layout).
template <typename T>
hipError_t xpass_T(const Ctx& c, const void* src, void* dst, const void* twx, unsigned long long* px, uint8_t* fmask) {
  const Plan& p = *c.p;
  const ColGeom g = geom_x(p, p.pitch, p.plane);
  if (c.pD)
    return run_col<T>(p.dt, COL_XPASSP, 0, g, p, src, dst, twx, c.st(), px, nullptr, c.s, nullptr, c.pD, g.so, g.s,
                      p.dt == FFCZ_F64 ? 1 : 0);
  return run_col<T>(p.dt, c.facc ? COL_XEDIT : COL_XPASS, c.facc ? 0 : p.vx, g, p, src, dst, twx, c.st(), px, fmask,
                    c.s, c.facc);
}

template <typename T>
hipError_t enqueue_round(const Ctx& c, int r, unsigned long long* viol, int64_t vstride, uint8_t* fmask,
                         uint32_t* smask) {
  const Plan& p = *c.p;
  unsigned long long* px = c.part(Ctx::PX);
  const char* twb = (const char*)c.twT();
  const void* twy = twb + sizeof(cx<T>) * p.twy;
  const void* twx = twb + sizeof(cx<T>) * p.twx;
  hipError_t e;
  if (p.nd == 3) {
    e = timed(PK_YFWD, r, c.s, [&] {
      return run_col<T>(p.dt, COL_FWD, p.vy, geom_y(p, p.pitch, p.plane), p, c.Z(), c.A(), twy, c.st(), px, fmask, c.s);
    });
    if (e != hipSuccess) return e;
    e = timed(PK_XPASS, r, c.s, [&] { return xpass_T<T>(c, c.A(), c.A(), twx, px, fmask); });
    if (e != hipSuccess) return e;
    e = launch_ctl(c, viol, vstride);
    if (e != hipSuccess) return e;
    e = timed(PK_YINV, r, c.s, [&] {
      return run_col<T>(p.dt, COL_INV, p.vy, geom_y(p, p.pitch, p.plane), p, c.A(), c.A(), twy, c.st(), px, fmask, c.s);
    });
    if (e != hipSuccess) return e;
  } else {
    e = timed(PK_XPASS, r, c.s, [&] { return xpass_T<T>(c, c.Z(), c.A(), twx, px, fmask); });
    if (e != hipSuccess) return e;
    e = launch_ctl(c, viol, vstride);
    if (e != hipSuccess) return e;
  }
  return timed(PK_ZPASS, r, c.s, [&] { return row_T<T>(ROW_LOOP, c, c.A(), c.Z(), smask); });
}

// The check that ends the loop (converged, or at the round cap) clips inside the x-pass, but
// that clip never reaches the iterate; with edit bookkeeping its displacements went into
// the frequency edits all the same.  Repeat that check's forward transforms from Z (which
// still holds the last-axis R2C of the checked iterate) and subtract the same displacements.
template <typename T>
hipError_t enqueue_undo(const Ctx& c) {
  const Plan& p = *c.p;
  const char* twb = (const char*)c.twT();
  const void* twy = twb + sizeof(cx<T>) * p.twy;
  const void* twx = twb + sizeof(cx<T>) * p.twx;
  if (p.nd == 3) {
    hipError_t e = run_col<T>(p.dt, COL_FWD_NS, 0, geom_y(p, p.pitch, p.plane), p, c.Z(), c.A(), twy, c.st(), nullptr,
                              nullptr, c.s);
    if (e != hipSuccess) return e;
    return run_col<T>(p.dt, COL_XUNDO, 0, geom_x(p, p.pitch, p.plane), p, c.A(), nullptr, twx, c.st(), nullptr,
                      nullptr, c.s, c.facc);
  }
  return run_col<T>(p.dt, COL_XUNDO, 0, geom_x(p, p.pitch, p.plane), p, c.Z(), nullptr, twx, c.st(), nullptr,
                    nullptr, c.s, c.facc);
}

// FP64 verification: last-axis R2C of y - x (max |y - x|), then the y and x
// transforms of that spectrum with the max-reduce in the x-pass.
template <typename T>
hipError_t enqueue_verify(const Ctx& c, bool z_done) {
  const Plan& p = *c.p;
  const char* tb = (const char*)c.tw64();
  void* W = c.W();
  hipError_t e = hipSuccess;
  if (!z_done) {
    e = timed(PK_VZ, -1, c.s, [&] {
      return run_row<double, T>(1, p.dt, c.pD ? ROW_VERIFYP : ROW_VERIFY, kVerifyRowPlan, p, p.pitch64, p.plane64,
                                nullptr, W, tb + 16 * (kVerifyRowPlan == 2 ? p.twz8 : p.twz), c.st(),
                                c.part(Ctx::PVZ), nullptr, c.s);
    });
    if (e != hipSuccess) return e;
  }
  if (p.nd == 3) {
    e = timed(PK_VY, -1, c.s, [&] {
      return run_col<double>(1, COL_FWD_NS, 0, geom_y(p, p.pitch64, p.plane64), p, W, W, tb + 16 * p.twy, c.st(),
                             c.part(Ctx::PVX), nullptr, c.s);
    });
    if (e != hipSuccess) return e;
  }
  e = timed(PK_VX, -1, c.s, [&] {
    if (c.pD) {
      // bounds at the working-type spectrum's layout, the transform at the FP64 one
      const ColGeom gb = geom_x(p, p.pitch, p.plane);
      return run_col<double>(1, COL_VERIFYP, 0, geom_x(p, p.pitch64, p.plane64), p, W, W, tb + 16 * p.twx, c.st(),
                             c.part(Ctx::PVX), nullptr, c.s, nullptr, c.pD, gb.so, gb.s, p.dt == FFCZ_F64 ? 1 : 0);
    }
    return run_col<double>(1, COL_VERIFY, 0, geom_x(p, p.pitch64, p.plane64), p, W, W, tb + 16 * p.twx, c.st(),
                           c.part(Ctx::PVX), nullptr, c.s);
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(stats_kernel, dim3((unsigned)p.B), dim3(1024), 0, c.s, c.st(), c.part(Ctx::PVZ), p.vzbpi,
                     c.part(Ctx::PVX), c.part(Ctx::PVX + 1), p.vxbpi);
  return hipGetLastError();
}

// Closing pass (y = x + eps, FP64 closing clamp) and, when asked, the FP64 verification.
template <typename T>
hipError_t enqueue_final(const Ctx& c, bool verify) {
  const Plan& p = *c.p;
  if (c.pD) {  // pointwise bounds: closing clamp against E_n, then the pointwise verification
    hipError_t e = timed(PK_FINAL, -1, c.s, [&] {
      return run_row<T, T>(p.dt, p.dt, ROW_FINALP, 0, p, p.pitch, p.plane, c.Z(), nullptr,
                           (const char*)c.twT() + sizeof(cx<T>) * p.twz, c.st(), c.part(Ctx::PZ), nullptr, c.s);
    });
    if (e != hipSuccess || !verify) return e;
    return enqueue_verify<T>(c, false);
  }
  if (!final_fused(p)) {
    hipError_t e = timed(PK_FINAL, -1, c.s, [&] { return row_T<T>(ROW_FINAL, c, c.Z(), nullptr, nullptr); });
    if (e != hipSuccess || !verify) return e;
    return enqueue_verify<T>(c, false);
  }
  const char* tb = (const char*)c.tw64();
  const int mode = verify ? ROW_FINALV : ROW_FINAL;
  hipError_t e = timed(PK_FINAL, -1, c.s, [&] {
    return run_row<double, T>(1, p.dt, mode, 2, p, p.pitch64, p.plane64, c.Z(), c.W(), tb + 16 * p.twz8, c.st(),
                              c.part(Ctx::PVZ), nullptr, c.s, p.pitch, p.plane);
  });
  if (e != hipSuccess || !verify) return e;
  return enqueue_verify<T>(c, true);
}

// pinned host staging (one per thread), grown on demand
struct HostBuf {
  void* p = nullptr;
  size_t n = 0;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t reserve(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) n = bytes;
    return e;
  }
};
thread_local HostBuf g_host_state, g_host_init, g_host_misc;
// staging of the 1D members (descriptors, then their loop states), owned by the calling
// thread and handed to the thread that drives those members, so that no pinned buffer is
// allocated or freed per call on a short-lived thread (hipHostFree synchronises the device)
thread_local HostBuf g_host_sig, g_host_sigstate;

// Private streams (default priority): one to capture graphs on, one for the
// 1D members of a batch, which run beside the grouped members.
struct Streams {
  // cap, cap2: capture (the second for a graph's parallel branch); side: the 1D members of a
  // mixed batch; side2: the 1D members that run one block each
  hipStream_t cap = nullptr, cap2 = nullptr, side = nullptr, side2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, fork2 = nullptr, join2 = nullptr, ready1d = nullptr, looped = nullptr,
             cfork = nullptr, cjoin = nullptr;
  ~Streams() {
    for (hipStream_t q : {cap, cap2, side, side2})
      if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t ev : {fork, join, fork2, join2, ready1d, looped, cfork, cjoin})
      if (ev) (void)hipEventDestroy(ev);
  }
  hipError_t ready() {
    hipError_t e = hipSuccess;
    for (hipStream_t* q : {&cap, &cap2, &side, &side2})
      if (e == hipSuccess && !*q) e = hipStreamCreateWithFlags(q, hipStreamNonBlocking);
    for (hipEvent_t* ev : {&fork, &join, &fork2, &join2, &ready1d, &looped, &cfork, &cjoin})
      if (e == hipSuccess && !*ev) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    return e;
  }
};
thread_local Streams g_streams;

// Instantiated graphs of a chunk of rounds, keyed by everything the launches capture.
struct GraphKey {
  std::vector<int64_t> k;
  bool operator<(const GraphKey& o) const { return k < o.k; }
};
struct GraphCache {
  std::map<GraphKey, hipGraphExec_t> m;
  std::vector<GraphKey> order;
  ~GraphCache() {
    for (auto& kv : m) (void)hipGraphExecDestroy(kv.second);
  }
  hipGraphExec_t find(const GraphKey& key) {
    auto it = m.find(key);
    return it == m.end() ? nullptr : it->second;
  }
  void put(const GraphKey& key, hipGraphExec_t g) {
    if (m.size() >= 16) {
      auto old = order.front();
      order.erase(order.begin());
      auto it = m.find(old);
      if (it != m.end()) {
        (void)hipGraphExecDestroy(it->second);
        m.erase(it);
      }
    }
    m[key] = g;
    order.push_back(key);
  }
};
thread_local GraphCache g_graphs;
// Graphs of the tiled 1D rounds: process-wide (the thread that drives the 1D members of a
// mixed batch is started per call), behind a mutex.  Never destroyed at exit: the HIP runtime
// may already be gone when static destructors run.
std::mutex g_sig_graphs_m;
GraphCache& sig_graphs() {
  static GraphCache* c = new GraphCache();
  return *c;
}

double bits_to_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, 8);
  return d;
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Plan tuner.  Each loop pass of a plan (y-forward/inverse, x-pass, last-axis
// pass) has a few variants: tilings that compute bit-identical results and
// differ only in how many columns / rows one block owns, and for the last-axis
// passes a radix-8 stage plan.  On the first use of a pass geometry on a device
// architecture, every variant is timed on the plan's own workspace (in place on
// the scratch spectrum, before the correction starts) and the fastest is kept;
// a variant other than the default must win by 2 % (rows) or 10 % (columns).
// The table is process-wide and, when a cache path is set, read from and
// written back to a JSON file.

struct TuneEntry {
  int choice = 0;
  std::vector<float> ms;
};

struct Tuner {
  std::mutex m;
  int mode = -1;  // -1: not read yet; 0: default plans; 1: tune on a miss; 2: narrower tiles; 3: radix-8 rows
  bool loaded = false;
  std::string path;
  std::map<std::string, TuneEntry> tab;

  void init_locked() {
    if (mode >= 0) return;
    const char* e = getenv("FFCZ_AUTOTUNE");
    mode = (e && e[0] == '0') ? 0 : 1;
    const char* c = getenv("FFCZ_PLAN_CACHE");
    if (c && *c) path = c;
  }
  // Entries are one per line: "key": {"choice": N, "ms": [..]}.  Lines that do
  // not parse are ignored, so a damaged file only costs a re-tune.
  void load_locked() {
    if (loaded) return;
    loaded = true;
    if (path.empty()) return;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return;
    char line[1024];
    while (fgets(line, sizeof(line), f)) {
      const char* q0 = strchr(line, '"');
      if (!q0) continue;
      const char* q1 = strchr(q0 + 1, '"');
      if (!q1) continue;
      const char* ch = strstr(q1, "\"choice\":");
      if (!ch) continue;
      int v = -1;
      if (sscanf(ch + 9, "%d", &v) != 1 || v < 0 || v >= std::max(kColVariants, kRowVariants)) continue;
      TuneEntry te;
      te.choice = v;
      tab[std::string(q0 + 1, q1)] = te;
    }
    fclose(f);
  }
  void save_locked() {
    if (path.empty()) return;
    const std::string tmp = path + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n \"format\": \"ffcz tile plans 1\",\n \"entries\": {\n");
    size_t i = 0;
    for (const auto& kv : tab) {
      fprintf(f, "  \"%s\": {\"choice\": %d, \"ms\": [", kv.first.c_str(), kv.second.choice);
      for (size_t k = 0; k < kv.second.ms.size(); ++k) fprintf(f, "%s%.5f", k ? ", " : "", kv.second.ms[k]);
      fprintf(f, "]}%s\n", ++i < tab.size() ? "," : "");
    }
    fprintf(f, " }\n}\n");
    const bool ok = fclose(f) == 0;
    if (ok) rename(tmp.c_str(), path.c_str());
  }
};
Tuner g_tuner;

std::string device_arch() {
  thread_local std::map<int, std::string> names;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  std::string n = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n = prop.gcnArchName;
  names[dev] = n;
  return n;
}

// The variant kept for `key`; on a miss, time `launch(v)` for every variant
// (only if may_time, else the default tiles).
template <typename F>
int32_t tune_pass(const std::string& key, hipStream_t s, bool may_time, float keep, int nvar, F&& launch, int* out) {
  *out = 0;
  {
    std::lock_guard<std::mutex> g(g_tuner.m);
    g_tuner.init_locked();
    g_tuner.load_locked();
    if (g_tuner.mode == 0) return FFCZ_OK;
    if (g_tuner.mode == 2) {  // the narrower tiles
      *out = 1;
      return FFCZ_OK;
    }
    if (g_tuner.mode == 3) {  // the radix-8 last-axis plan
      *out = nvar > 2 ? 2 : 0;
      return FFCZ_OK;
    }
    if (g_tuner.mode == 4) {  // the direct (index-fastest) last-axis loop pass
      *out = nvar > 3 ? 3 : 0;
      return FFCZ_OK;
    }
    auto it = g_tuner.tab.find(key);
    if (it != g_tuner.tab.end() && it->second.choice < nvar) {
      *out = it->second.choice;
      return FFCZ_OK;
    }
  }
  if (!may_time) return FFCZ_OK;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  TuneEntry te;
  hipError_t err = hipSuccess;
  for (int v = 0; v < nvar && err == hipSuccess; ++v) {
    err = launch(v);  // warm-up
    if (err != hipSuccess) break;
    float best = 1e30f;
    for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
      err = hipEventRecord(e0, s);
      if (err == hipSuccess) err = launch(v);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms);
    }
    te.ms.push_back(best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(err);
  te.choice = 0;
  for (int v = 1; v < nvar; ++v)
    if (te.ms[v] < keep * te.ms[0] && te.ms[v] < te.ms[te.choice]) te.choice = v;
  std::lock_guard<std::mutex> g(g_tuner.m);
  g_tuner.tab[key] = te;
  g_tuner.save_locked();
  *out = te.choice;
  return FFCZ_OK;
}

// A narrower column tile reads 64-byte halves of lines whose other halves belong to
// another block (fetched again, from the last-level cache at best), so it must win clearly.
constexpr float kColKeep = 0.90f;

// Pick the loop passes' tile variants for plan p (state and twiddles already
// written; the scratch spectrum A is overwritten).  Nothing is timed while the
// stream is being captured or masks are recorded (the loop kernels would write
// mask planes); mask recording also keeps the default x-pass tiles, whose
// width the 1-bit mask words assume.
// Table key of a plan's last-axis loop pass.
std::string tune_key_z(const Plan& p) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%s z H=%d rows=%lld", (device_arch() + (p.dt == FFCZ_F32 ? " f32" : " f64")).c_str(), p.H,
           (long long)(p.nrows * p.B));
  return buf;
}

// no_time: take the table's decisions (or the defaults) without timing anything.
template <typename T>
int32_t tune_plan(Plan& p, char* ws, hipStream_t s, bool rec, bool no_time = false) {
  const std::string pre = device_arch() + (p.dt == FFCZ_F32 ? " f32" : " f64");
  char buf[256];
  int vy = 0, vx = 0, vz = 0;
  Ctx c{&p, ws, s};
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(s, &cs));
  const bool may_time = !rec && !no_time && cs == hipStreamCaptureStatusNone;
  const char* twb = (const char*)c.twT();
  if (p.nd == 3 && p.Ly >= 64) {
    snprintf(buf, sizeof(buf), "%s y L=%d cols=%lld outer=%lld", pre.c_str(), p.Ly, (long long)p.ncols,
             (long long)p.n[0]);
    int32_t r = tune_pass(buf, s, may_time, kColKeep, kColVariants, [&](int v) {
      return run_col<T>(p.dt, COL_FWD, v, geom_y(p, p.pitch, p.plane), p, c.A(), c.A(), twb + sizeof(cx<T>) * p.twy,
                        c.st(), c.part(Ctx::PX), nullptr, s);
    }, &vy);
    if (r != FFCZ_OK) return r;
  }
  if (p.nd >= 2 && p.Lx >= 64 && !rec) {
    snprintf(buf, sizeof(buf), "%s x L=%d cols=%lld outer=%lld B=%lld", pre.c_str(), p.Lx, (long long)p.ncols,
             (long long)(p.nd == 3 ? p.n[1] : 1), (long long)p.B);
    int32_t r = tune_pass(buf, s, may_time, kColKeep, kColVariants, [&](int v) {
      Plan q = p;
      set_variants(q, q.vy, v, q.vz);
      return run_col<T>(p.dt, COL_XPASS, v, geom_x(q, q.pitch, q.plane), q, c.A(), c.A(), twb + sizeof(cx<T>) * p.twx,
                        c.st(), c.part(Ctx::PX), nullptr, s);
    }, &vx);
    if (r != FFCZ_OK) return r;
  }
  if (p.H >= 64) {
    int32_t r = tune_pass(tune_key_z(p), s, may_time, 0.98f, kRowVariants, [&](int v) {
      return run_row<T, T>(p.dt, p.dt, ROW_LOOP, v, p, p.pitch, p.plane, c.A(), c.A(),
                           twb + sizeof(cx<T>) * (v == 2 ? p.twz8 : p.twz), c.st(),
                           c.part(Ctx::PZ), nullptr, s);
    }, &vz);
    if (r != FFCZ_OK) return r;
  }
  set_variants(p, vy, vx, vz);
  return FFCZ_OK;
}

// Tune a group's passes ahead of a mixed batch, before the 1D members start on
// the side stream (their work would disturb the timings): a neutral state (loop
// not done, no masks) and the twiddles are written, then tune_plan runs on the
// group's own workspace.  The decisions land in the process-wide table.
template <typename T>
int32_t pretune_group(const Plan& p0, char* ws, hipStream_t s) {
  Plan p = p0;
  Ctx c{&p, ws, s};
  StateInit one;
  memset(&one, 0, sizeof(one));
  one.max_iter = 1;
  hipLaunchKernelGGL(state_init_kernel, dim3((unsigned)std::max<int64_t>(1, (p.B + 255) / 256)), dim3(256), 0, s,
                     c.st(), p.B, (const StateInit*)nullptr, one, (unsigned long long*)nullptr, (int64_t)0);
  HIPCHK(hipGetLastError());
  HIPCHK(write_twiddles(c));
  return tune_plan<T>(p, ws, s, false);
}

// Edit bookkeeping of an encoder call (null for a plain correction).
struct EditCfg {
  void* sacc;     // spatial accumulators: N values of the working type, C order
  void* facc;     // frequency accumulators: laid out as the spectrum Z
  bool derive;    // shrinks from x on the device; else mu_s / mu_f below
  double q;       // safety 2^-m (derive)
  double mu_s, mu_f;
  bool want_y;    // close y = x + eps (and verify it when asked)
  unsigned long long* amax;  // kUlpSlots partial slots of max |x| (derive)
  double* mu_s_out;          // host: the spatial shrink in use, read back with the state
};

// Workspace of the encoder and decoder: the plan's, then the accumulators and the
// coding kernels' block offsets.
struct EditLayout {
  int64_t ncs = 0, ncf = 0;  // spatial and frequency coordinates
  int64_t nbs = 0, nbf = 0;  // coding blocks of each set
  size_t off_S = 0, off_F = 0, off_offs = 0, off_offf = 0, off_tot = 0, off_amax = 0, bytes = 0;
  int64_t spec_reals = 0;    // working-type reals of one spectrum buffer (padding included)
};

EditLayout edit_layout(const Plan& p) {
  EditLayout L;
  const size_t ts = p.dt == FFCZ_F32 ? 4 : 8;
  L.ncs = p.N * p.B;
  L.ncf = 2 * p.nrows * p.ncols * p.B;
  L.nbs = (L.ncs + kEditBlockCoords - 1) / kEditBlockCoords;
  L.nbf = (L.ncf + kEditBlockCoords - 1) / kEditBlockCoords;
  const int64_t rpp = p.nd == 3 ? p.n[1] : p.nrows;
  L.spec_reals = 2 * p.B * (p.nrows / rpp) * p.plane;
  size_t off = align_up(p.bytes, 256);
  L.off_S = off;
  off = align_up(off + ts * (size_t)L.ncs, 256);
  L.off_F = off;
  off = align_up(off + ts * (size_t)L.spec_reals, 256);
  L.off_offs = off;
  off = align_up(off + 8 * (size_t)std::max<int64_t>(1, L.nbs), 256);
  L.off_offf = off;
  off = align_up(off + 8 * (size_t)std::max<int64_t>(1, L.nbf), 256);
  L.off_tot = off;  // two totals and the status word
  off = align_up(off + 8 * 4, 256);
  L.off_amax = off;
  off = align_up(off + 8 * (size_t)kUlpSlots, 256);
  L.bytes = off;
  return L;
}

// Pointwise bounds of a ffcz_correct_bounds call (null for scalar bounds).
struct BoundsCfg {
  const void* pE;               // E_n (caller's device array, field dtype) or null: the scalar E
  const void* dre;              // D^Re_k (or the disk's D_k), half-spectrum C order, or null
  const void* dim;              // D^Im_k or null (then D^Re_k, or the scalar)
  double sre, sim;              // scalar spectral bounds where the arrays are null
  int disk;
  void* pD;                     // workspace: the bound pairs laid out as the spectrum
  unsigned long long* minpart;  // workspace: kMinSlots block minima
  unsigned long long* bad;      // workspace: invalid-entry counter
};

// Workspace of ffcz_correct_bounds and ffcz_power_spectrum_bounds beyond the plan's: the bound
// pairs, block minima and a counter; for the power-spectrum bound a zero field (the verification
// pass transforms y - x, here x - 0), the per-block shell sums and the shell bounds.
struct BoundsLayout {
  size_t off_D = 0, off_min = 0, off_bad = 0, off_zero = 0, off_shell = 0, off_bins = 0, bytes = 0;
  int nb = 0;   // shells
  int nsb = 0;  // shell-sum blocks
};

BoundsLayout bounds_layout(const Plan& p) {
  BoundsLayout L;
  const size_t ts = p.dt == FFCZ_F32 ? 4 : 8;
  double kmax2 = 0.0;
  for (int i = 0; i < p.nd; ++i) kmax2 += (double)(p.n[i] / 2) * (double)(p.n[i] / 2);
  L.nb = (int)std::lrint(std::sqrt(kmax2)) + 1;
  const int64_t M = p.nrows * p.ncols;
  L.nsb = (int)std::max<int64_t>(1, std::min<int64_t>(256, (M + 4095) / 4096));
  const int64_t rpp = p.nd == 3 ? p.n[1] : p.nrows;
  size_t off = align_up(p.bytes, 256);
  L.off_D = off;
  off = align_up(off + 2 * ts * (size_t)(p.nrows / rpp) * (size_t)p.plane, 256);
  L.off_min = off;
  off = align_up(off + 8 * (size_t)kMinSlots, 256);
  L.off_bad = off;
  off = align_up(off + 8, 256);
  L.off_zero = off;
  off = align_up(off + ts * (size_t)p.N, 256);
  L.off_shell = off;
  off = align_up(off + 8 * 3 * (size_t)L.nsb * (size_t)L.nb, 256);
  L.off_bins = off;
  off = align_up(off + 8 * (size_t)L.nb, 256);
  L.bytes = off;
  return L;
}

// One correction over the B instances of a plan.  inst[b] supplies pointers and
// bounds, mus[b] the margins; mus null (one FP32 instance) derives mu from x on
// the device, between the state set-up and the first pass.
// host_state: when given (one entry per instance, ordinary host memory), the call
// allocates nothing: the loop state is read back into it, the rounds run as plain
// launches (no graph) and the tile plans come from the table or the defaults.
// One group's correction (a plan over B same-shape instances) in phases: begin (set-up through
// the first last-axis transform, on the call's stream), the rounds in chunks (run here, or
// captured with other work by the mixed-batch loop), end (closing pass, verification,
// statistics).  Holds a Ctx that points at its own Plan: neither copied nor moved.
template <typename T>
struct GroupRun {
  Plan p;
  Ctx c{nullptr, nullptr, nullptr};
  const ffcz_instance* inst = nullptr;
  const double* mus = nullptr;
  int32_t max_iter = 0;
  ffcz_options o{};
  DevState* host_state = nullptr;  // the no-allocation form's host copy of the state (else null)
  const EditCfg* ed = nullptr;
  const BoundsCfg* bc = nullptr;
  bool no_alloc = false, rec = false;
  unsigned long long* viol = nullptr;
  int64_t vstr = 0;
  uint32_t* smask = nullptr;
  uint8_t* fmask = nullptr;
  int chunk = 4;

  GroupRun() = default;
  GroupRun(const GroupRun&) = delete;
  GroupRun& operator=(const GroupRun&) = delete;

  int32_t begin(const Plan& p0, const ffcz_instance* inst_, const double* mus_, int32_t max_iter_,
                const ffcz_options& o_, char* ws, hipStream_t s, DevState* host_state_, const EditCfg* ed_,
                const BoundsCfg* bc_) {
    inst = inst_;
    mus = mus_;
    max_iter = max_iter_;
    o = o_;
    host_state = host_state_;
    ed = ed_;
    bc = bc_;
    no_alloc = host_state != nullptr;
    p = p0;
    c = Ctx{&p, ws, s};
    if (ed) {
      c.sacc = ed->sacc;
      c.facc = ed->facc;
    }
    if (bc) c.pD = bc->pD;
    const int64_t vstride = max_iter + 2;
    const bool user_viol = o.viol_per_round && p.B == 1;
    viol = user_viol ? (unsigned long long*)o.viol_per_round : c.viol();
    vstr = user_viol ? 0 : vstride;
    rec = o.masks_out != nullptr && p.B == 1;
    smask = rec ? (uint32_t*)o.masks_out : nullptr;
    fmask = rec ? (uint8_t*)o.masks_out + (size_t)(max_iter + 1) * p.s_plane_bytes : nullptr;
    chunk = o.graph_chunk > 0 ? o.graph_chunk : 4;

    auto fill = [&](int64_t b) {
      StateInit si;
      memset(&si, 0, sizeof(si));
      si.E = inst[b].eps_s;
      const double mu = mus ? mus[b] : 0.0;  // without mus, margin_kernel rewrites the mu-dependent fields
      si.Ep = inst[b].eps_s * (1.0 - mu);
      si.Delta = inst[b].delta_f;
      spectral_thresholds(p.dt, inst[b].delta_f, mu, &si.Dc, &si.Dp);
      si.inv_n = 1.0 / (double)p.N;
      si.mu = mu;
      if (ed && !ed->derive) {  // the encoder's given shrinks
        si.mu = ed->mu_f;
        si.mu_s = ed->mu_s;
        si.Ep = inst[b].eps_s * (1.0 - ed->mu_s);
        si.Dc = inst[b].delta_f * (1.0 - ed->mu_f);
        si.Dp = inst[b].delta_f * (1.0 - 2.0 * ed->mu_f);
      }
      if (bc) {
        si.pE = bc->pE;
        si.pD = bc->pD;
        si.disk = bc->disk;
      }
      si.max_iter = max_iter;
      si.fixed = o.fixed_iterations ? 1 : 0;
      si.record_masks = rec ? 1 : 0;
      si.px = inst[b].x_orig;
      si.pxb = inst[b].x_base;
      si.py = inst[b].x_out;
      return si;
    };
    const StateInit* arr = nullptr;
    StateInit one = fill(0);
    if (p.B > 1) {
      HIPCHK(g_host_init.reserve(sizeof(StateInit) * p.B));
      StateInit* h = (StateInit*)g_host_init.p;
      for (int64_t b = 0; b < p.B; ++b) h[b] = fill(b);
      arr = (const StateInit*)(ws + p.off_init);
      HIPCHK(hipMemcpyAsync((void*)arr, h, sizeof(StateInit) * p.B, hipMemcpyHostToDevice, s));
    }
    const int64_t nviol = user_viol ? (int64_t)max_iter + 1 : vstride * p.B;
    const int64_t nthr = std::max<int64_t>(p.B, nviol);
    hipLaunchKernelGGL(state_init_kernel, dim3((unsigned)std::max<int64_t>(1, (nthr + 255) / 256)), dim3(256), 0, s,
                       c.st(), p.B, arr, one, viol, nviol);
    HIPCHK(hipGetLastError());
    if (bc) {
      // the bound pairs into the spectrum layout, their checks and minimum, then mu and the factors
      if (p.B != 1) return fail(FFCZ_E_INVALID, "pointwise bounds take one instance");
      hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, bc->bad, (int64_t)1);
      HIPCHK(hipGetLastError());
      const int64_t M = p.nrows * p.ncols;
      const int nmin = (int)std::max<int64_t>(1, std::min<int64_t>(kMinSlots, (M + 255) / 256));
      const SpecGeom g{p.nrows, (int32_t)p.ncols, p.lg_rpp, p.pitch, p.plane};
      hipLaunchKernelGGL(bounds_setup_kernel<T>, dim3((unsigned)nmin), dim3(256), 0, s, (const T*)bc->dre,
                         (const T*)bc->dim, bc->sre, bc->sim, (cx<T>*)bc->pD, M, g, bc->minpart, bc->bad);
      HIPCHK(hipGetLastError());
      if (bc->pE) {
        const int nbe = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (p.N + 255) / 256));
        hipLaunchKernelGGL(spatial_check_kernel<T>, dim3((unsigned)nbe), dim3(256), 0, s, (const T*)bc->pE, p.N,
                           bc->bad);
        HIPCHK(hipGetLastError());
      }
      double* slots = (double*)(ws + p.off_ulp);
      const double mu_given = mus ? mus[0] : 0.0;
      if (p.dt == FFCZ_F32 && !(mu_given > 0.0)) {
        const MarginJob one_job{(const float*)inst[0].x_orig, p.N, 0.0};
        hipLaunchKernelGGL(ulp_part_kernel, dim3((unsigned)ulp_slots(p.N)), dim3(256), 0, s, one_job,
                           (const MarginJob*)nullptr, slots);
        HIPCHK(hipGetLastError());
      }
      hipLaunchKernelGGL(bounds_margin_kernel, dim3(1), dim3(256), 0, s, (const double*)slots,
                         (const unsigned long long*)bc->minpart, nmin, p.N, (int)p.dt, bc->disk, mu_given, c.st());
      HIPCHK(hipGetLastError());
      unsigned long long nbad = 0;
      HIPCHK(hipMemcpyAsync(&nbad, bc->bad, sizeof(nbad), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (nbad) return fail(FFCZ_E_INVALID, "bound arrays must hold finite values >= 0 (" + std::to_string(nbad) +
                                                " entries do not)");
    } else if (ed && ed->derive) {
      // the encoder's shrinks from x (ulp partials for the FP32 output margin, max |x|)
      if (p.B != 1) return fail(FFCZ_E_INVALID, "the encoder takes one instance");
      const int nsl = ulp_slots(p.N);
      double* slots = (double*)(ws + p.off_ulp);
      if (p.dt == FFCZ_F32) {
        const MarginJob one_job{(const float*)inst[0].x_orig, p.N, inst[0].delta_f};
        hipLaunchKernelGGL(ulp_part_kernel, dim3((unsigned)nsl), dim3(256), 0, s, one_job, (const MarginJob*)nullptr,
                           slots);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(absmax_part_kernel<float>, dim3((unsigned)nsl), dim3(256), 0, s,
                           (const float*)inst[0].x_orig, p.N, ed->amax);
      } else {
        hipLaunchKernelGGL(absmax_part_kernel<double>, dim3((unsigned)nsl), dim3(256), 0, s,
                           (const double*)inst[0].x_orig, p.N, ed->amax);
      }
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(encode_margin_kernel, dim3(1), dim3(256), 0, s, (const double*)slots,
                         (const unsigned long long*)ed->amax, p.N, (int)p.dt, ed->q, c.st());
      HIPCHK(hipGetLastError());
    } else if (!mus) {
      if (p.B != 1 || p.dt != FFCZ_F32) return fail(FFCZ_E_INVALID, "device margin needs one FP32 instance");
      const int nsl = ulp_slots(p.N);
      double* slots = (double*)(ws + p.off_ulp);
      const MarginJob one_job{(const float*)inst[0].x_orig, p.N, inst[0].delta_f};
      hipLaunchKernelGGL(ulp_part_kernel, dim3((unsigned)nsl), dim3(256), 0, s, one_job, (const MarginJob*)nullptr,
                         slots);
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(margin_kernel, dim3(1), dim3(256), 0, s, (const double*)slots, one_job,
                         (const MarginJob*)nullptr, (int)p.dt, (double*)nullptr, c.st());
      HIPCHK(hipGetLastError());
    }
    HIPCHK(write_twiddles(c));
    if (bc) {
      set_variants(p, 0, 0, 0);  // the pointwise passes exist for the default tiles only
    } else if (ed) {
      // edit bookkeeping runs on the default tiles; the frequency accumulators start at zero
      set_variants(p, 0, 0, 0);
      const int64_t nr = edit_layout(p).spec_reals;
      hipLaunchKernelGGL(zero_fill_kernel<T>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, (T*)ed->facc, nr);
      HIPCHK(hipGetLastError());
    } else {
      const int32_t tr = tune_plan<T>(p, ws, s, rec, no_alloc);
      if (tr != FFCZ_OK) return tr;
    }
    HIPCHK(timed(PK_INIT, -1, s, [&] { return row_T<T>(ROW_INIT, c, nullptr, c.Z(), smask); }));
    return FFCZ_OK;
  }

  // One chunk of rounds on st (the round passes return at entry once the instance is done).
  hipError_t enqueue_chunk(hipStream_t st) const {
    Ctx cc{&p, c.ws, st};
    cc.sacc = c.sacc;
    cc.facc = c.facc;
    cc.pD = c.pD;
    for (int r = 0; r < chunk; ++r) {
      const hipError_t e = enqueue_round<T>(cc, r, viol, vstr, fmask, smask);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // Everything a captured chunk bakes in.
  GraphKey graph_key() const {
    return GraphKey{{(int64_t)p.dt, p.nd, p.B, p.n[0], p.n[1], p.n[2], (int64_t)(uintptr_t)c.ws,
                     (int64_t)(uintptr_t)viol, vstr, (int64_t)(uintptr_t)fmask, (int64_t)(uintptr_t)smask, chunk,
                     max_iter, p.vy, p.vx, p.vz, (int64_t)(uintptr_t)c.sacc, (int64_t)(uintptr_t)c.facc,
                     (int64_t)(uintptr_t)c.pD}};
  }

  // The host copy of the instances' states (the no-allocation form brings its own).
  int32_t host_states(DevState** hs) {
    if (!no_alloc) HIPCHK(g_host_state.reserve(sizeof(DevState) * p.B));
    *hs = no_alloc ? host_state : (DevState*)g_host_state.p;
    return FFCZ_OK;
  }

  // The rounds, driven from here: fixed rounds enqueued at once, else chunks (captured once in
  // a hipGraph unless per-launch timing is on) with one poll of the done-flags per chunk.
  int32_t loop() {
    const hipStream_t s = c.s;
    DevState* hs = nullptr;
    int32_t hr = host_states(&hs);
    if (hr != FFCZ_OK) return hr;
    if (o.fixed_iterations) {
      // exactly max_iter blocks plus the final check: no polling needed
      for (int r = 0; r <= max_iter; ++r) HIPCHK(enqueue_round<T>(c, r, viol, vstr, fmask, smask));
      return FFCZ_OK;
    }
    hipGraphExec_t gexec = nullptr;
    if (o.use_graph && !g_prof.on && !no_alloc) {
      const GraphKey key = graph_key();
      gexec = g_graphs.find(key);
      if (!gexec) {
        HIPCHK(g_streams.ready());
        HIPCHK(hipStreamBeginCapture(g_streams.cap, hipStreamCaptureModeThreadLocal));
        const hipError_t ce = enqueue_chunk(g_streams.cap);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(g_streams.cap, &graph);
        if (ce != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          return fail(FFCZ_E_HIP, std::string("capture: ") + hipGetErrorString(ce));
        }
        HIPCHK(ee);
        const hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ie);
        g_graphs.put(key, gexec);
      }
    }
    for (int enq = 0;;) {
      if (gexec) HIPCHK(hipGraphLaunch(gexec, s));
      else
        for (int r = 0; r < chunk; ++r) HIPCHK(enqueue_round<T>(c, enq + r, viol, vstr, fmask, smask));
      enq += chunk;
      HIPCHK(hipMemcpyAsync(hs, c.st(), sizeof(DevState) * p.B, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bool all = true;
      for (int64_t b = 0; b < p.B; ++b) all = all && hs[b].done;
      if (all) break;
      if (enq > max_iter + 2 * chunk + 2)
        return fail(FFCZ_E_HIP, "loop did not report completion (device state inconsistent)");
    }
    return FFCZ_OK;
  }

  // After the rounds: the closing pass and verification, then (unless nothing is reported)
  // the instances' statistics and statuses.
  int32_t end(ffcz_stats* stats, int32_t* status) {
    DevState* hs = nullptr;
    int32_t hr = host_states(&hs);
    if (hr != FFCZ_OK) return hr;
    // asynchronous only when nothing is reported: fixed rounds, no statistics, no verification
    const bool sync_needed = !(o.fixed_iterations && stats == nullptr && !o.verify_fp64);
    if (ed) HIPCHK(enqueue_undo<T>(c));
    if (!ed || ed->want_y) HIPCHK(enqueue_final<T>(c, o.verify_fp64 != 0));
    if (!sync_needed) {
      prof_settle(max_iter);
      for (int64_t b = 0; b < p.B; ++b) status[b] = FFCZ_OK;
      return FFCZ_OK;
    }
    HIPCHK(hipMemcpyAsync(hs, c.st(), sizeof(DevState) * p.B, hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipStreamSynchronize(c.s));
    int maxr = 0;
    for (int64_t b = 0; b < p.B; ++b) maxr = std::max(maxr, hs[b].round);
    prof_settle(maxr);
    if (ed && ed->mu_s_out) *ed->mu_s_out = hs[0].mu_s;
    for (int64_t b = 0; b < p.B; ++b) {
      const DevState& h = hs[b];
      const double ms = bits_to_double(h.max_spatial_bits), mf = bits_to_double(h.max_spectral_bits);
      if (stats) {
        ffcz_stats& st = stats[b];
        memset(&st, 0, sizeof(st));
        st.rounds = h.round;
        st.converged = h.converged;
        st.f_viol_initial = (int64_t)h.v_first;
        st.f_viol_final = (int64_t)h.v_last;
        st.s_clipped_total = (int64_t)h.s_clipped_total;
        st.s_guard = (int64_t)h.s_guard;
        st.nonfinite = (int64_t)h.nonfinite;
        st.max_spatial_err = o.verify_fp64 ? ms : NAN;
        st.max_spectral_err = o.verify_fp64 ? mf : NAN;
        st.spectral_viol = (int64_t)h.spectral_viol;
        st.margin_used = h.mu;
      }
      int32_t r = FFCZ_OK;
      if (h.nonfinite) r = FFCZ_E_NONFINITE;
      else if (!h.converged && !o.fixed_iterations) r = FFCZ_NOT_CONVERGED;
      else if (o.verify_fp64 && bc && (!(ms <= 1.0) || !(mf <= 1.0) || h.spectral_viol)) r = FFCZ_VERIFY_FAILED;
      else if (o.verify_fp64 && !bc && (!(ms <= inst[b].eps_s) || !(mf <= inst[b].delta_f))) r = FFCZ_VERIFY_FAILED;
      status[b] = r;
    }
    return FFCZ_OK;
  }
};

template <typename T>
int32_t correct_group(const Plan& p0, const ffcz_instance* inst, const double* mus, int32_t max_iter,
                      const ffcz_options& o, char* ws, hipStream_t s, ffcz_stats* stats, int32_t* status,
                      DevState* host_state = nullptr, const EditCfg* ed = nullptr,
                      const BoundsCfg* bc = nullptr) {
  GroupRun<T> g;
  int32_t r = g.begin(p0, inst, mus, max_iter, o, ws, s, host_state, ed, bc);
  if (r != FFCZ_OK) return r;
  r = g.loop();
  if (r != FFCZ_OK) return r;
  return g.end(stats, status);
}

template <typename T>
int32_t backward_impl(const Plan& p, int32_t rounds, const void* masks, const void* gy, void* gb, void* ws,
                      hipStream_t s) {
  Ctx c{&p, (char*)ws, s};
  StateInit si;
  memset(&si, 0, sizeof(si));
  si.inv_n = 1.0 / (double)p.N;
  si.max_iter = rounds;
  si.pxb = gy;
  si.py = gb;
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, c.st(), (int64_t)1, (const StateInit*)nullptr, si,
                     c.viol(), (int64_t)1);
  HIPCHK(hipGetLastError());
  HIPCHK(write_twiddles(c));
  const char* mb = (const char*)masks;
  auto splane = [&](int k) { return (uint32_t*)(mb + (size_t)k * p.s_plane_bytes); };
  auto fplane = [&](int k) {
    return (uint8_t*)(mb + (size_t)(rounds + 1) * p.s_plane_bytes + (size_t)(k - 1) * 2 * p.f_plane_bytes);
  };
  const char* twb = (const char*)c.twT();
  const void* twy = twb + sizeof(cx<T>) * p.twy;
  const void* twx = twb + sizeof(cx<T>) * p.twx;
  if (rounds == 0) {
    // y = x + M_s^0 (x_hat - x): the gradient is the guard mask times dL/dy (applied twice; masks are idempotent)
    HIPCHK(row_T<T>(ROW_BINIT, c, nullptr, c.Z(), splane(0)));
    HIPCHK(row_T<T>(ROW_BFINAL, c, c.Z(), nullptr, splane(0)));
    return FFCZ_OK;
  }
  HIPCHK(timed(PK_BZ, -1, s, [&] { return row_T<T>(ROW_BINIT, c, nullptr, c.Z(), splane(rounds)); }));
  for (int k = rounds; k >= 1; --k) {
    if (p.nd == 3)
      HIPCHK(timed(PK_BY, -1, s, [&] {
        return run_col<T>(p.dt, COL_FWD_NS, 0, geom_y(p, p.pitch, p.plane), p, c.Z(), c.Z(), twy, c.st(), nullptr, nullptr, s);
      }));
    HIPCHK(timed(PK_BX, -1, s, [&] {
      return run_col<T>(p.dt, COL_XBACK, 0, geom_x(p, p.pitch, p.plane), p, c.Z(), c.Z(), twx, c.st(), nullptr, fplane(k), s);
    }));
    if (p.nd == 3)
      HIPCHK(timed(PK_BY, -1, s, [&] {
        return run_col<T>(p.dt, COL_INV_NS, 0, geom_y(p, p.pitch, p.plane), p, c.Z(), c.Z(), twy, c.st(), nullptr, nullptr, s);
      }));
    if (k > 1) HIPCHK(timed(PK_BZ, -1, s, [&] { return row_T<T>(ROW_BLOOP, c, c.Z(), c.Z(), splane(k - 1)); }));
    else HIPCHK(timed(PK_BZ, -1, s, [&] { return row_T<T>(ROW_BFINAL, c, c.Z(), nullptr, splane(0)); }));
  }
  return FFCZ_OK;
}

// ---------------------------------------------------------------------------
// 1D batch members: one block per signal (kernels_sig.hpp)


struct SigPlan {
  int dt = 0;
  int64_t L = 0;
  int blue = 0;
  int lgMc = 0;
  size_t conv64 = 0, btab = 0, btab64 = 0, btabi = 0, chirp = 0, chirp64 = 0, eps = 0, bytes = 0;  // offsets in the signal block
};

SigPlan sig_plan(int dt, int64_t L) {
  SigPlan s;
  s.dt = dt;
  s.L = L;
  s.blue = (is_pow2(L) && L >= 4) ? 0 : 1;  // direct four-step needs Mc = L >= 4
  // Bluestein over the half spectrum: Mc >= L + K - 1 with K = floor(L/2) + 1
  s.lgMc = s.blue ? ceil_lg(L + L / 2) : ceil_lg(L);
  if (s.lgMc < 2) s.lgMc = 2;
  const size_t Mc = (size_t)1 << s.lgMc;
  size_t off = 0;
  s.conv64 = off;
  off = align_up(off + 16 * Mc, 256);
  if (s.blue) {
    s.btab64 = off;
    off = align_up(off + 16 * Mc, 256);
    s.chirp64 = off;
    off = align_up(off + 16 * (size_t)L, 256);
    if (dt == FFCZ_F32) {
      s.btab = off;
      off = align_up(off + 8 * Mc, 256);
      s.chirp = off;
      off = align_up(off + 8 * (size_t)L, 256);
    } else {
      s.btab = s.btab64;
      s.chirp = s.chirp64;
    }
    s.btabi = off;  // the reflected table, in the loop's working type
    off = align_up(off + (dt == FFCZ_F32 ? 8 : 16) * Mc, 256);
  }
  s.eps = off;
  off = align_up(off + (dt == FFCZ_F32 ? 4 : 8) * (size_t)L, 256);
  s.bytes = off;
  return s;
}

// four-step tables of one convolution length: working type and FP64, both layouts
struct McTabs {
  size_t tw4, tw4r, twa, twb, tw4_64, tw4r_64, twa_64, twb_64, bytes;
};

int sig_ma(int lgMc) { return 1 << ((lgMc + 1) / 2); }

McTabs mc_tabs(int dt, int lgMc) {
  const int MA = sig_ma(lgMc), MB = (1 << lgMc) / MA;
  const size_t Mc = (size_t)1 << lgMc;
  const size_t cs = dt == FFCZ_F32 ? 8 : 16;
  McTabs t;
  size_t off = 0;
  t.tw4 = off;
  off = align_up(off + cs * Mc, 256);
  t.tw4r = off;
  off = align_up(off + cs * Mc, 256);
  t.twa = off;
  off = align_up(off + cs * (host_twsize(MA, pick_E(MA)) + 1), 256);
  t.twb = off;
  off = align_up(off + cs * (host_twsize(MB, pick_E(MB)) + 1), 256);
  t.tw4_64 = off;
  off = align_up(off + 16 * Mc, 256);
  t.tw4r_64 = off;
  off = align_up(off + 16 * Mc, 256);
  t.twa_64 = off;
  off = align_up(off + 16 * (host_twsize(MA, pick_E(MA)) + 1), 256);
  t.twb_64 = off;
  off = align_up(off + 16 * (host_twsize(MB, pick_E(MB)) + 1), 256);
  t.bytes = off;
  return t;
}

// W_Mc^{n1 k2} in the column layout [k2][n1] and in the row-pass layout of the sig kernel
__global__ void tw4_kernel(void* col, void* row, int dbl, int lgMc, int MA, int RR) {
  const int64_t Mc = (int64_t)1 << lgMc;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mc) return;
  const int64_t k2 = i / MA, n1 = i % MA;
  const int64_t r = (n1 * k2) & (Mc - 1);
  double sn, cs;
  sincospi(-2.0 * (double)r / (double)Mc, &sn, &cs);
  const int64_t rp = ((k2 / RR) * MA + n1) * RR + (k2 % RR);
  if (dbl) {
    ((cx<double>*)col)[i] = cx<double>{cs, sn};
    ((cx<double>*)row)[rp] = cx<double>{cs, sn};
  } else {
    ((cx<float>*)col)[i] = cx<float>{__double2float_rn(cs), __double2float_rn(sn)};
    ((cx<float>*)row)[rp] = cx<float>{__double2float_rn(cs), __double2float_rn(sn)};
  }
}

hipError_t write_mc_tabs(int dt, int lgMc, char* base, const McTabs& t, hipStream_t s) {
  const int MA = sig_ma(lgMc), MB = (1 << lgMc) / MA;
  const int64_t Mc = (int64_t)1 << lgMc;
  for (int pass = 0; pass < 2; ++pass) {
    const int dbl = (pass == 1 || dt == FFCZ_F64) ? 1 : 0;
    char* col = base + (pass ? t.tw4_64 : t.tw4);
    char* row = base + (pass ? t.tw4r_64 : t.tw4r);
    hipLaunchKernelGGL(tw4_kernel, dim3((unsigned)((Mc + 255) / 256)), dim3(256), 0, s, col, row, dbl, lgMc, MA,
                       sig_rows_per_tile(dbl, lgMc));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TwJobs ja, jb;
    memset(&ja, 0, sizeof(ja));
    ja.dbl = dbl;
    ja.n = 1;
    jb = ja;
    ja.j[0] = TwJob{0, MA, pick_E(MA), 0};
    jb.j[0] = TwJob{0, MB, pick_E(MB), 0};
    hipLaunchKernelGGL(twiddle_kernel, dim3(64, 2), dim3(256), 0, s, (void*)(base + (pass ? t.twa_64 : t.twa)), ja,
                       (void*)(base + (pass ? t.twb_64 : t.twb)), jb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Layout of the batched workspace

struct BatchPlan {
  int dt = 0;
  std::vector<int> sig_ids;                 // 1D members
  std::vector<SigPlan> sigs;
  std::map<int, std::vector<int>> by_mc;    // lgMc -> positions in sig_ids
  std::map<int, size_t> mc_off;             // lgMc -> table offset
  std::map<int, McTabs> mc_tab;
  std::vector<size_t> sig_off;
  size_t off_desc = 0, off_sstats = 0, off_order = 0, off_mjobs = 0, off_msum = 0;
  // length classes run as tiled passes: partial slots [kind][signal][tile] per class
  std::map<int, size_t> tpart_off;
  std::map<int, int> tpart_tiles;
  // multi-dimensional groups
  std::vector<std::vector<int>> groups;
  std::vector<Plan> gplans;
  std::vector<size_t> goff;
  size_t bytes = 0;
};

int32_t batch_plan(int32_t dt, int32_t count, const ffcz_instance* inst, int32_t max_iter, BatchPlan& bp) {
  bp = BatchPlan();
  bp.dt = dt;
  if (dt != FFCZ_F32 && dt != FFCZ_F64) return fail(FFCZ_E_INVALID, "dtype must be FFCZ_F32 or FFCZ_F64");
  if (count < 0 || (count > 0 && !inst)) return fail(FFCZ_E_INVALID, "bad instance array");
  std::map<std::vector<int64_t>, int> gkey;
  for (int i = 0; i < count; ++i) {
    const ffcz_instance& in = inst[i];
    if (in.ndim < 1 || in.ndim > 3) return fail(FFCZ_E_SHAPE, "instance ndim must be 1..3");
    int64_t sq[3];
    for (int d = 0; d < in.ndim; ++d)
      if (in.shape[d] < 1) return fail(FFCZ_E_SHAPE, "every extent must be >= 1");
    const int nd = squeeze(in.ndim, in.shape, sq);
    if (nd <= 1) {
      const int64_t L = nd == 0 ? 1 : sq[0];
      if (L > (int64_t)1 << 19) return fail(FFCZ_E_SHAPE, "1D lengths must be at most 2^19");
      bp.sig_ids.push_back(i);
      continue;
    }
    std::vector<int64_t> key(sq, sq + nd);
    if (nd == 3) key.push_back(i);  // 3D instances run one at a time
    auto it = gkey.find(key);
    if (it == gkey.end()) {
      gkey[key] = (int)bp.groups.size();
      bp.groups.push_back({i});
    } else {
      bp.groups[it->second].push_back(i);
    }
  }
  size_t off = 0;
  for (auto& g : bp.groups) {
    Plan p;
    const ffcz_instance& in = inst[g[0]];
    int32_t r = make_plan(dt, in.ndim, in.shape, max_iter, (int64_t)g.size(), p);
    if (r != FFCZ_OK) return r;
    bp.gplans.push_back(p);
    bp.goff.push_back(off);
    off = align_up(off + p.bytes, 256);
  }
  const int ns = (int)bp.sig_ids.size();
  for (int k = 0; k < ns; ++k) {
    int64_t sq[3];
    const ffcz_instance& in = inst[bp.sig_ids[k]];
    const int nd = squeeze(in.ndim, in.shape, sq);
    SigPlan sp = sig_plan(dt, nd == 0 ? 1 : sq[0]);
    bp.sigs.push_back(sp);
    bp.by_mc[sp.lgMc].push_back(k);
    bp.sig_off.push_back(off);
    off = align_up(off + sp.bytes, 256);
  }
  for (auto& kv : bp.by_mc) {
    McTabs t = mc_tabs(dt, kv.first);
    bp.mc_tab[kv.first] = t;
    bp.mc_off[kv.first] = off;
    off = align_up(off + t.bytes, 256);
  }
  for (auto& kv : bp.by_mc) {
    if (kv.first < kSigTiledMinLg) continue;  // partial slots for every class that may run tiled
    int nct = 0, nrt = 0;
    sig_tiles(kv.first, &nct, &nrt);
    const int pt = std::max(nct, nrt);
    bp.tpart_off[kv.first] = off;
    bp.tpart_tiles[kv.first] = pt;
    off = align_up(off + sizeof(unsigned long long) * SP_KINDS * kv.second.size() * (size_t)pt, 256);
  }
  bp.off_desc = off;
  off = align_up(off + sizeof(SigDesc) * (size_t)std::max(ns, 1), 256);
  bp.off_sstats = off;
  off = align_up(off + sizeof(SigStats) * (size_t)std::max(ns, 1), 256);
  bp.off_order = off;
  off = align_up(off + sizeof(int32_t) * (size_t)std::max(ns, 1), 256);
  bp.off_mjobs = off;  // margin jobs (x pointer, length, bound)
  off = align_up(off + sizeof(MarginJob) * (size_t)std::max(count, 1), 256);
  bp.off_msum = off;  // margin partial sums (kUlpSlots per member), then the members' mu
  off = align_up(off + sizeof(double) * (size_t)(kUlpSlots + 1) * (size_t)std::max(count, 1), 256);
  bp.bytes = off;
  return FFCZ_OK;
}

// Tiled loop control, one block per signal slot of a length class: sum the
// check's partial counts (and the spatial-clip counts of the pass that made the
// checked iterate), record them, and decide whether the signal's loop ends.
__global__ void __launch_bounds__(256) sig_ctl_kernel(const SigDesc* sig, SigStats* stats, const int32_t* order,
                                                       const unsigned long long* part, int32_t nsig, int32_t ptiles,
                                                       int32_t nct, int32_t nrt, int32_t max_iter, int32_t fixed) {
  __shared__ unsigned long long red[3][4];
  const int slot = blockIdx.x;
  if (slot >= nsig) return;
  const int sid = order[slot];
  SigStats* so = stats + sid;
  if (*(volatile int32_t*)&so->done) return;
  const int nck = sig[sid].blue ? nct : nrt;  // tiles of the pass that counted violations
  const int k = so->rounds;
  auto at = [&](int kind, int tl) { return part[((int64_t)kind * nsig + slot) * ptiles + tl]; };
  unsigned long long v = 0, z = 0, nf = 0;
  for (int i = threadIdx.x; i < nck; i += blockDim.x) v += at(SP_VIOL, i);
  for (int i = threadIdx.x; i < nct; i += blockDim.x) {
    z += at(SP_SCLIP, i);
    if (k == 0) nf += at(SP_NONFIN, i);
  }
  v = wave_sum_u64(v);
  z = wave_sum_u64(z);
  nf = wave_sum_u64(nf);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = v;
    red[1][threadIdx.x >> 6] = z;
    red[2][threadIdx.x >> 6] = nf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long V = 0, Z = 0, NF = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
      V += red[0][w];
      Z += red[1][w];
      NF += red[2][w];
    }
    if (k == 0) {
      so->s_guard = Z;
      so->viol0 = V;
    } else {
      so->s_clipped += Z;
    }
    so->violf = V;
    int stop = 0;
    if (k == 0 && NF) {
      so->nonfinite = NF;
      so->nonfinite_stop = 1;
      so->converged = 0;
      stop = 1;
    } else if (!fixed && V == 0) {
      so->converged = 1;
      stop = 1;
    } else if (k >= max_iter) {
      so->converged = (V == 0) ? 1 : 0;
      stop = 1;
    }
    if (stop) so->done = 1;
    else so->rounds = k + 1;
  }
}

// Tiled verification totals, one block per signal slot.
__global__ void __launch_bounds__(256) sig_vstats_kernel(const SigDesc* sig, SigStats* stats, const int32_t* order,
                                                          const unsigned long long* part, int32_t nsig, int32_t ptiles,
                                                          int32_t nct, int32_t nrt) {
  __shared__ unsigned long long red[3][4];
  const int slot = blockIdx.x;
  if (slot >= nsig) return;
  const int sid = order[slot];
  SigStats* so = stats + sid;
  const int nv = sig[sid].blue ? nct : nrt;
  auto at = [&](int kind, int tl) { return part[((int64_t)kind * nsig + slot) * ptiles + tl]; };
  unsigned long long mf = 0, ms = 0, c = 0;  // maxima of non-negative doubles compare as their bits
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    const unsigned long long b = at(SP_VMAXF, i);
    mf = mf > b ? mf : b;
    c += at(SP_VCNT, i);
  }
  for (int i = threadIdx.x; i < nct; i += blockDim.x) {
    const unsigned long long b = at(SP_VMAXS, i);
    ms = ms > b ? ms : b;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o1 = __shfl_xor(mf, off, 64), o2 = __shfl_xor(ms, off, 64);
    mf = mf > o1 ? mf : o1;
    ms = ms > o2 ? ms : o2;
    c += __shfl_xor(c, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = mf;
    red[1][threadIdx.x >> 6] = ms;
    red[2][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long F = 0, S = 0, C = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
      F = F > red[0][w] ? F : red[0][w];
      S = S > red[1][w] ? S : red[1][w];
      C += red[2][w];
    }
    so->max_spectral = __longlong_as_double((long long)F);
    so->max_spatial = __longlong_as_double((long long)S);
    so->spectral_viol = C;
  }
}

template <typename T>
hipError_t sig_launch(int dt, int mode, int lgMc, const BatchPlan& bp, char* ws, const int32_t* order,
                      int nsig, int32_t max_iter, int32_t fixed, hipStream_t s) {
  const McTabs& t = bp.mc_tab.at(lgMc);
  char* tb = ws + bp.mc_off.at(lgMc);
  const bool d64 = sig_mode_fp64(mode, dt);
  SigArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.sig = (const SigDesc*)(ws + bp.off_desc);
  a.stats = (SigStats*)(ws + bp.off_sstats);
  a.order = order;
  a.nsig = nsig;
  a.max_iter = max_iter;
  a.fixed = fixed;
  a.tab.tw4 = (const cx<T>*)(tb + (d64 ? t.tw4_64 : t.tw4));
  a.tab.tw4r = (const cx<T>*)(tb + (d64 ? t.tw4r_64 : t.tw4r));
  a.tab.twa = (const cx<T>*)(tb + (d64 ? t.twa_64 : t.twa));
  a.tab.twb = (const cx<T>*)(tb + (d64 ? t.twb_64 : t.twb));
  auto it = bp.tpart_off.find(lgMc);
  if (it != bp.tpart_off.end()) {
    a.part = (unsigned long long*)(ws + it->second);
    a.ptiles = bp.tpart_tiles.at(lgMc);
  }
  return launch_sig(dt, mode, lgMc, &a, nsig, s);
}

// Descriptors (bounds, thresholds, buffer addresses) and block order of the 1D members, and
// the four-step tables of every length class; first[lg] is the class's first slot in the order.
int32_t sig_prepare(const BatchPlan& bp, const ffcz_instance* inst, const double* mus, char* ws, hipStream_t s,
                    HostBuf& hsig, std::map<int, int>& first) {
  const int ns = (int)bp.sig_ids.size();
  // own staging buffer: the grouped members reuse g_host_init while these copies may be in flight
  HIPCHK(hsig.reserve(sizeof(SigDesc) * ns + sizeof(int32_t) * ns));
  SigDesc* hd = (SigDesc*)hsig.p;
  int32_t* ho = (int32_t*)(hd + ns);
  for (int k = 0; k < ns; ++k) {
    const ffcz_instance& in = inst[bp.sig_ids[k]];
    const SigPlan& sp = bp.sigs[k];
    char* b = ws + bp.sig_off[k];
    SigDesc d;
    memset(&d, 0, sizeof(d));
    d.x = in.x_orig;
    d.xb = in.x_base;
    d.y = in.x_out;
    d.L = sp.L;
    d.blue = sp.blue;
    d.E = in.eps_s;
    d.Delta = in.delta_f;
    d.Ep = in.eps_s * (1.0 - mus[bp.sig_ids[k]]);
    spectral_thresholds(bp.dt, in.delta_f, mus[bp.sig_ids[k]], &d.Dc, &d.Dp);
    d.conv = b + sp.conv64;
    d.conv64 = b + sp.conv64;
    if (sp.blue) {
      d.btab = b + sp.btab;
      d.btab64 = b + sp.btab64;
      d.btabi = b + sp.btabi;
      d.chirp = b + sp.chirp;
      d.chirp64 = b + sp.chirp64;
    }
    d.eps = b + sp.eps;
    hd[k] = d;
  }
  // block order per convolution length: larger signals first
  int pos = 0;
  first.clear();
  for (auto& kv : bp.by_mc) {
    std::vector<int> ids = kv.second;
    std::sort(ids.begin(), ids.end(), [&](int a, int b) { return bp.sigs[a].L > bp.sigs[b].L; });
    first[kv.first] = pos;
    for (int id : ids) ho[pos++] = id;
  }
  HIPCHK(hipMemcpyAsync(ws + bp.off_desc, hd, sizeof(SigDesc) * ns, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + bp.off_order, ho, sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
  for (auto& kv : bp.by_mc)
    HIPCHK(write_mc_tabs(bp.dt, kv.first, ws + bp.mc_off.at(kv.first), bp.mc_tab.at(kv.first), s));
  return FFCZ_OK;
}

// One-block or tiled for a length class.  A threshold given in the options decides alone;
// otherwise classes below 2^kSigTiledMinLg run one block per signal, classes above 2^16 run
// tiled, and the ones between take the tuner's decision for (architecture, data type, work
// length, power-of-two bucket of the class's signal count, kinds of length): variant 0 is the
// default rule (tiled from 2^15), variant 1 the other form.
constexpr int kSigTuneMaxLg = 16;
std::string sig_tune_key(const BatchPlan& bp, int lg) {
  const std::vector<int>& ids = bp.by_mc.at(lg);
  int n = 1;
  while (n < (int)ids.size()) n <<= 1;
  bool blue = false, p2 = false;
  for (int k : ids) (bp.sigs[k].blue ? blue : p2) = true;
  char buf[160];
  snprintf(buf, sizeof(buf), "%s %s sig lg=%d n<=%d kinds=%s%s", device_arch().c_str(),
           bp.dt == FFCZ_F32 ? "f32" : "f64", lg, n, blue ? "b" : "", p2 ? "p" : "");
  return buf;
}
bool sig_default_tiled(int lg) { return lg >= 15; }

// The decision for class lg without timing (the table's entry, else the default rule).
int32_t sig_class_tiled(const BatchPlan& bp, const ffcz_options& o, int lg, hipStream_t s, bool* tiled) {
  if (o.tiled_1d_lg > 0) {
    *tiled = lg >= std::max(kSigTiledMinLg, (int)o.tiled_1d_lg);
    return FFCZ_OK;
  }
  if (lg < kSigTiledMinLg || lg > kSigTuneMaxLg) {
    *tiled = lg >= kSigTiledMinLg;
    return FFCZ_OK;
  }
  int v = 0;
  int32_t r = tune_pass(sig_tune_key(bp, lg), s, false, 0.9f, 2, [](int) { return hipSuccess; }, &v);
  if (r != FFCZ_OK) return r;
  *tiled = sig_default_tiled(lg) != (v == 1);
  return FFCZ_OK;
}

// A class's correction with a fixed number of rounds and no verification, one-block or tiled:
// the timing run of the tuner (writes the members' outputs, which the real run rewrites).
template <typename T>
hipError_t sig_trial(const BatchPlan& bp, char* ws, const int32_t* ord, int lg, bool tiled, bool resident,
                     int rounds, hipStream_t s) {
  const int nb = (int)bp.by_mc.at(lg).size();
  const int ns = (int)bp.sig_ids.size();
  auto go = [&](int mode) -> hipError_t {
    if (sig_mode_fp64(mode, bp.dt)) return sig_launch<double>(bp.dt, mode, lg, bp, ws, ord, nb, rounds, 1, s);
    return sig_launch<T>(bp.dt, mode, lg, bp, ws, ord, nb, rounds, 1, s);
  };
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((ns * sizeof(SigStats) / 8 + 255) / 256)), dim3(256), 0, s,
                     (unsigned long long*)(ws + bp.off_sstats), (int64_t)(ns * sizeof(SigStats) / 8));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!tiled) {
    if ((e = go(SIG_SETUP)) != hipSuccess) return e;
    return go(resident && sig_res_fits(bp.dt, lg) ? SIG_RUNL : SIG_RUN);
  }
  bool blue = false, p2 = false;
  for (int k : bp.by_mc.at(lg)) (bp.sigs[k].blue ? blue : p2) = true;
  if (blue)
    for (int m : {(int)SIGT_CHIRP, (int)SIGT_BCOL, (int)SIGT_BROW})
      if ((e = go(m)) != hipSuccess) return e;
  if ((e = go(SIGT_EPS0)) != hipSuccess) return e;
  if ((e = go(SIGT_CIN)) != hipSuccess) return e;
  int nct = 0, nrt = 0;
  sig_tiles(lg, &nct, &nrt);
  for (int r = 0; r <= rounds; ++r) {  // fixed rounds: the control stops the loop at the last check
    if (blue && (e = go(SIGT_RMUL)) != hipSuccess) return e;
    if (p2 && (e = go(SIGT_RCHECK)) != hipSuccess) return e;
    if (blue && (e = go(SIGT_CCHECK)) != hipSuccess) return e;
    hipLaunchKernelGGL(sig_ctl_kernel, dim3((unsigned)nb), dim3(256), 0, s, (const SigDesc*)(ws + bp.off_desc),
                       (SigStats*)(ws + bp.off_sstats), ord, (const unsigned long long*)(ws + bp.tpart_off.at(lg)),
                       (int32_t)nb, (int32_t)bp.tpart_tiles.at(lg), (int32_t)nct, (int32_t)nrt, (int32_t)rounds,
                       (int32_t)1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (blue && (e = go(SIGT_RMULI)) != hipSuccess) return e;
    if ((e = go(SIGT_CSPAT)) != hipSuccess) return e;
  }
  return go(SIGT_Y);
}

// Time both forms of every class the tuner decides and has no entry for, on the call's own
// members (three fixed rounds each, before the real run; nothing else runs meanwhile).
int32_t pretune_sigs(const BatchPlan& bp, const ffcz_instance* inst, const double* mus, const ffcz_options& o,
                     char* ws, hipStream_t s, HostBuf& hsig) {
  if (bp.sig_ids.empty() || o.tiled_1d_lg > 0) return FFCZ_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return FFCZ_OK;  // nothing is timed under capture
  std::map<int, int> first;
  bool prepared = false;
  for (auto& kv : bp.by_mc) {
    const int lg = kv.first;
    if (lg < kSigTiledMinLg || lg > kSigTuneMaxLg) continue;
    if (!prepared) {
      int32_t r = sig_prepare(bp, inst, mus, ws, s, hsig, first);
      if (r != FFCZ_OK) return r;
      prepared = true;
    }
    const int32_t* ord = (const int32_t*)(ws + bp.off_order) + first[lg];
    const bool dflt = sig_default_tiled(lg);
    int v = 0;
    int32_t r = tune_pass(sig_tune_key(bp, lg), s, true, 0.9f, 2, [&](int var) {
      const bool tiled = dflt != (var == 1);
      return bp.dt == FFCZ_F32 ? sig_trial<float>(bp, ws, ord, lg, tiled, o.resident_1d != 0, 3, s)
                               : sig_trial<double>(bp, ws, ord, lg, tiled, o.resident_1d != 0, 3, s);
    }, &v);
    if (r != FFCZ_OK) return r;
  }
  return FFCZ_OK;
}

// The 1D members of a batch in phases: begin (descriptors and tables, the one-block classes on
// their own stream, the tiled classes' set-up), the tiled rounds in chunks (run here, or
// captured with the groups' rounds by the mixed-batch loop), end (the tiled classes' outputs and
// verification, then the one-block stream joined).  Every tiled round pass returns at entry once
// its signal's loop has ended.
struct SigRun {
  const BatchPlan* bp = nullptr;
  const ffcz_instance* inst = nullptr;
  const double* mus = nullptr;
  int32_t max_iter = 0;
  ffcz_options o{};
  char* ws = nullptr;
  hipStream_t s = nullptr;       // set-up, tiled passes, end
  hipStream_t side = nullptr;    // one-block classes (joined into s at the end)
  hipEvent_t fork = nullptr, join = nullptr;
  std::map<int, int> first;      // class -> first slot in the block order
  std::vector<int> tiled;
  std::map<int, std::pair<bool, bool>> kinds;  // class -> (has Bluestein lengths, has power-of-two lengths)
  int fixed = 0, chunk = 4;
  bool side_used = false;

  const int32_t* order() const { return (const int32_t*)(ws + bp->off_order); }
  int nsig() const { return (int)bp->sig_ids.size(); }

  // a launch of one mode over every signal of class lg, in the mode's arithmetic, on st
  hipError_t go(int mode, int lg, hipStream_t st) const {
    const int nb = (int)bp->by_mc.at(lg).size();
    const int32_t* ord = order() + first.at(lg);
    if (sig_mode_fp64(mode, bp->dt)) return sig_launch<double>(bp->dt, mode, lg, *bp, ws, ord, nb, max_iter, fixed, st);
    return sig_launch<float>(bp->dt, mode, lg, *bp, ws, ord, nb, max_iter, fixed, st);
  }

  int32_t begin(const BatchPlan& bp_, const ffcz_instance* inst_, const double* mus_, int32_t max_iter_,
                const ffcz_options& o_, char* ws_, hipStream_t s_, hipStream_t side_, hipEvent_t fork_,
                hipEvent_t join_, HostBuf& hsig) {
    bp = &bp_;
    inst = inst_;
    mus = mus_;
    max_iter = max_iter_;
    o = o_;
    ws = ws_;
    s = s_;
    side = side_;
    fork = fork_;
    join = join_;
    fixed = o.fixed_iterations ? 1 : 0;
    chunk = o.graph_chunk > 0 ? o.graph_chunk : 4;
    const int ns = nsig();
    if (ns == 0) return FFCZ_OK;
    int32_t pr = sig_prepare(*bp, inst, mus, ws, s, hsig, first);
    if (pr != FFCZ_OK) return pr;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((ns * sizeof(SigStats) / 8 + 255) / 256)), dim3(256), 0, s,
                       (unsigned long long*)(ws + bp->off_sstats), (int64_t)(ns * sizeof(SigStats) / 8));
    HIPCHK(hipGetLastError());
    std::vector<int> oneblock;
    for (auto& kv : bp->by_mc) {
      const int lg = kv.first;
      bool is_tiled = false;
      int32_t tr = sig_class_tiled(*bp, o, lg, s, &is_tiled);
      if (tr != FFCZ_OK) return tr;
      if (!is_tiled) {
        oneblock.push_back(lg);
        continue;
      }
      tiled.push_back(lg);
      bool b = false, p2 = false;
      for (int k : kv.second) (bp->sigs[k].blue ? b : p2) = true;
      kinds[lg] = {b, p2};
    }
    // the one-block classes run their whole correction on their own stream, beside the tiled
    // rounds (and, in a mixed batch, beside the grouped members: the set-up's end on s does
    // not wait for them)
    hipStream_t sb = s;
    if (!oneblock.empty() && side) {
      HIPCHK(hipEventRecord(fork, s));
      HIPCHK(hipStreamWaitEvent(side, fork, 0));
      sb = side;
      side_used = true;
    }
    for (int lg : oneblock) {
      HIPCHK(go(SIG_SETUP, lg, sb));
      HIPCHK(go(o.resident_1d && sig_res_fits(bp->dt, lg) ? SIG_RUNL : SIG_RUN, lg, sb));
      if (o.verify_fp64) HIPCHK(go(SIG_VERIFY, lg, sb));
    }
    // tiled classes: set-up, eps0 and the first forward column pass
    for (int lg : tiled) {
      if (kinds[lg].first) {
        HIPCHK(go(SIGT_CHIRP, lg, s));
        HIPCHK(go(SIGT_BCOL, lg, s));
        HIPCHK(go(SIGT_BROW, lg, s));
      }
      HIPCHK(go(SIGT_EPS0, lg, s));
      HIPCHK(go(SIGT_CIN, lg, s));
    }
    return FFCZ_OK;
  }

  // one chunk of rounds of every tiled class, on st
  hipError_t enqueue_chunk(hipStream_t st) const {
    hipError_t e = hipSuccess;
    for (int r = 0; r < chunk && e == hipSuccess; ++r) {
      for (int lg : tiled) {
        const bool b = kinds.at(lg).first, p2 = kinds.at(lg).second;
        if (b && (e = go(SIGT_RMUL, lg, st)) != hipSuccess) return e;
        if (p2 && (e = go(SIGT_RCHECK, lg, st)) != hipSuccess) return e;
        if (b && (e = go(SIGT_CCHECK, lg, st)) != hipSuccess) return e;
        int nct = 0, nrt = 0;
        sig_tiles(lg, &nct, &nrt);
        const int nb = (int)bp->by_mc.at(lg).size();
        hipLaunchKernelGGL(sig_ctl_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const SigDesc*)(ws + bp->off_desc),
                           (SigStats*)(ws + bp->off_sstats), order() + first.at(lg),
                           (const unsigned long long*)(ws + bp->tpart_off.at(lg)), (int32_t)nb,
                           (int32_t)bp->tpart_tiles.at(lg), (int32_t)nct, (int32_t)nrt, max_iter, (int32_t)fixed);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (b && (e = go(SIGT_RMULI, lg, st)) != hipSuccess) return e;
        if ((e = go(SIGT_CSPAT, lg, st)) != hipSuccess) return e;
      }
    }
    return e;
  }

  // everything a captured chunk bakes in: the workspace, the members' layout, the cap, the chunk
  void key_into(GraphKey& key) const {
    key.k.insert(key.k.end(), {-1, (int64_t)bp->dt, (int64_t)(uintptr_t)ws, (int64_t)max_iter, (int64_t)fixed,
                               (int64_t)chunk, (int64_t)nsig()});
    for (int k = 0; k < nsig(); ++k) {
      key.k.push_back(bp->sigs[k].L);
      key.k.push_back(bp->sigs[k].blue);
      key.k.push_back((int64_t)bp->sig_off[k]);
    }
    for (int lg : tiled) key.k.push_back(lg);
  }

  // whether every tiled signal's loop has ended, from a host copy of the signal states
  bool all_done(const SigStats* hs) const {
    for (int lg : tiled)
      for (int k : bp->by_mc.at(lg))
        if (!hs[k].done) return false;
    return true;
  }

  // the tiled rounds driven from here: chunks captured once in a hipGraph (process-wide cache)
  // and replayed, one poll of the done-flags per chunk
  int32_t loop(HostBuf& hstate) {
    if (tiled.empty()) return FFCZ_OK;
    const int ns = nsig();
    HIPCHK(hstate.reserve(sizeof(SigStats) * ns));
    SigStats* hs = (SigStats*)hstate.p;
    hipGraphExec_t gexec = nullptr;
    if (o.use_graph && !g_prof.on) {
      GraphKey key;
      key_into(key);
      std::lock_guard<std::mutex> lk(g_sig_graphs_m);
      gexec = sig_graphs().find(key);
      if (!gexec) {
        HIPCHK(g_streams.ready());
        HIPCHK(hipStreamBeginCapture(g_streams.cap, hipStreamCaptureModeThreadLocal));
        const hipError_t ce = enqueue_chunk(g_streams.cap);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(g_streams.cap, &graph);
        if (ce != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          return fail(FFCZ_E_HIP, std::string("capture of the 1D rounds: ") + hipGetErrorString(ce));
        }
        HIPCHK(ee);
        const hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ie);
        sig_graphs().put(key, gexec);
      }
    }
    for (int enq = 0;; enq += chunk) {
      if (gexec) HIPCHK(hipGraphLaunch(gexec, s));
      else HIPCHK(enqueue_chunk(s));
      HIPCHK(hipMemcpyAsync(hs, ws + bp->off_sstats, sizeof(SigStats) * ns, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (all_done(hs)) break;
      if (enq > max_iter + 2 * chunk + 2) return fail(FFCZ_E_HIP, "tiled signals did not report completion");
    }
    return FFCZ_OK;
  }

  // the tiled classes' outputs and verification on s, then s waits for the one-block classes
  int32_t end() {
    for (int lg : tiled) {
      HIPCHK(go(SIGT_Y, lg, s));
      if (!o.verify_fp64) continue;
      HIPCHK(go(SIGT_VCOL, lg, s));
      HIPCHK(go(SIGT_VROW, lg, s));
      if (kinds[lg].first) HIPCHK(go(SIGT_VCOL2, lg, s));
      int nct = 0, nrt = 0;
      sig_tiles(lg, &nct, &nrt);
      const int nb = (int)bp->by_mc.at(lg).size();
      hipLaunchKernelGGL(sig_vstats_kernel, dim3((unsigned)nb), dim3(256), 0, s, (const SigDesc*)(ws + bp->off_desc),
                         (SigStats*)(ws + bp->off_sstats), order() + first.at(lg),
                         (const unsigned long long*)(ws + bp->tpart_off.at(lg)), (int32_t)nb,
                         (int32_t)bp->tpart_tiles.at(lg), (int32_t)nct, (int32_t)nrt);
      HIPCHK(hipGetLastError());
    }
    return rejoin();
  }

  // s waits for the one-block stream (also on early exits, so no launch outlives the call)
  int32_t rejoin() {
    if (!side_used) return FFCZ_OK;
    side_used = false;
    HIPCHK(hipEventRecord(join, side));
    HIPCHK(hipStreamWaitEvent(s, join, 0));
    return FFCZ_OK;
  }
  ~SigRun() { (void)rejoin(); }
};

int32_t run_sigs(const BatchPlan& bp, const ffcz_instance* inst, const double* mus, int32_t max_iter,
                 const ffcz_options& o, char* ws, hipStream_t s, HostBuf& hsig, HostBuf& hstate) {
  if (bp.sig_ids.empty()) return FFCZ_OK;
  HIPCHK(g_streams.ready());
  SigRun sr;
  int32_t r = sr.begin(bp, inst, mus, max_iter, o, ws, s, g_streams.side2, g_streams.fork2, g_streams.join2, hsig);
  if (r != FFCZ_OK) return r;
  r = sr.loop(hstate);
  if (r != FFCZ_OK) return r;
  return sr.end();
}

int32_t collect_sigs(const BatchPlan& bp, const ffcz_instance* inst, const double* mus, const ffcz_options& o,
                     char* ws, hipStream_t s, ffcz_stats* stats, int32_t* status) {
  const int ns = (int)bp.sig_ids.size();
  if (ns == 0) return FFCZ_OK;
  HIPCHK(g_host_misc.reserve(sizeof(SigStats) * ns));
  SigStats* h = (SigStats*)g_host_misc.p;
  HIPCHK(hipMemcpyAsync(h, ws + bp.off_sstats, sizeof(SigStats) * ns, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < ns; ++k) {
    const int id = bp.sig_ids[k];
    const SigStats& g = h[k];
    if (stats) {
      ffcz_stats& st = stats[id];
      memset(&st, 0, sizeof(st));
      st.rounds = g.rounds;
      st.converged = g.converged;
      st.f_viol_initial = (int64_t)g.viol0;
      st.f_viol_final = (int64_t)g.violf;
      st.s_clipped_total = (int64_t)g.s_clipped;
      st.s_guard = (int64_t)g.s_guard;
      st.nonfinite = (int64_t)g.nonfinite;
      st.max_spatial_err = o.verify_fp64 ? g.max_spatial : NAN;
      st.max_spectral_err = o.verify_fp64 ? g.max_spectral : NAN;
      st.spectral_viol = (int64_t)g.spectral_viol;
      st.margin_used = mus[id];
    }
    int32_t r = FFCZ_OK;
    if (g.nonfinite_stop) r = FFCZ_E_NONFINITE;
    else if (!g.converged && !o.fixed_iterations) r = FFCZ_NOT_CONVERGED;
    else if (o.verify_fp64 && (!(g.max_spatial <= inst[id].eps_s) || !(g.max_spectral <= inst[id].delta_f)))
      r = FFCZ_VERIFY_FAILED;
    status[id] = r;
  }
  return FFCZ_OK;
}

// Streaming copy: one 16-byte vector per lane, one block per 4 KiB (measured on
// MI355X as the fastest of the simple forms: more work per lane or a grid-stride
// loop keeps fewer requests in flight).
__global__ void __launch_bounds__(256) copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                   int64_t n16) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

__global__ void copy_tail_kernel(unsigned char* __restrict__ dst, const unsigned char* __restrict__ src, int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

// Copy with the access pattern of the strided-axis passes: block (f, tile) moves the
// 128-byte tile of the rows (f, i) for every i along the axis, 16 bytes per lane, 8 lanes
// per tile row and 32 rows per step.  Row (f, i) starts at f fixed_stride + i axis_stride.
__global__ void __launch_bounds__(256) copy_columns_kernel(char* __restrict__ dst, const char* __restrict__ src,
                                                           int64_t n_axis, int64_t axis_stride, int64_t fixed_stride,
                                                           int64_t row_bytes, int32_t tiles) {
  const int64_t b = blockIdx.x;
  const int64_t f = b / tiles;
  const int tile = (int)(b - f * tiles);
  const int64_t off = (int64_t)tile * 128 + (threadIdx.x & 7) * 16;
  if (off >= row_bytes) return;  // row_bytes is a multiple of 16; no barrier follows
  const int64_t base = f * fixed_stride + off;
#pragma unroll 4
  for (int64_t i = threadIdx.x >> 3; i < n_axis; i += 32) {
    const int64_t a = base + i * axis_stride;
    *reinterpret_cast<uint4*>(dst + a) = *reinterpret_cast<const uint4*>(src + a);
  }
}

// Makes the caller's stream wait for the side stream on every exit after the fork, so no
// 1D launch still writes the caller's buffers once the call has returned.
struct SideJoin {
  hipStream_t s = nullptr, s1 = nullptr;
  ~SideJoin() {
    if (s1 && s1 != s) {
      (void)hipEventRecord(g_streams.join, s1);
      (void)hipStreamWaitEvent(s, g_streams.join, 0);
    }
  }
};


// A batch of 1D and grouped members, driven from the calling thread.  Everything is tuned
// first, with nothing else running.  Then the 1D set-up runs on a side stream (its one-block
// classes on a second one, beside everything else) while the groups' set-up runs on the caller's
// stream; every chunk of rounds is one hipGraph holding each group's chunk and every tiled 1D
// class's chunk as two parallel branches, replayed with one poll of all done-flags per chunk;
// last, the groups' closing passes on the caller's stream and the tiled classes' outputs and
// verification on the side stream, joined before return.
template <typename T>
int32_t mixed_batch(const BatchPlan& bp, const ffcz_instance* inst, const std::vector<double>& mus,
                    int32_t max_iter, const ffcz_options& o, char* w, hipStream_t s, ffcz_stats* stats,
                    std::vector<int32_t>& status) {
  for (size_t g = 0; g < bp.groups.size(); ++g) {
    int32_t r = pretune_group<T>(bp.gplans[g], w + bp.goff[g], s);
    if (r != FFCZ_OK) return r;
  }
  int32_t r = pretune_sigs(bp, inst, mus.data(), o, w, s, g_host_sig);
  if (r != FFCZ_OK) return r;
  HIPCHK(g_streams.ready());
  const hipStream_t s1 = g_streams.side;
  HIPCHK(hipEventRecord(g_streams.fork, s));
  HIPCHK(hipStreamWaitEvent(s1, g_streams.fork, 0));
  SideJoin side;  // s waits for s1 on every exit from here
  side.s = s;
  side.s1 = s1;
  SigRun sr;      // declared after the join: its own stream joins s1 first
  r = sr.begin(bp, inst, mus.data(), max_iter, o, w, s1, g_streams.side2, g_streams.fork2, g_streams.join2, g_host_sig);
  if (r != FFCZ_OK) return r;
  HIPCHK(hipEventRecord(g_streams.ready1d, s1));
  // the groups' set-up on s; their instance and margin arrays live as long as the runs
  const size_t ng = bp.groups.size();
  std::vector<std::vector<ffcz_instance>> gis(ng);
  std::vector<std::vector<double>> gms(ng);
  std::vector<std::unique_ptr<GroupRun<T>>> gr;
  for (size_t g = 0; g < ng; ++g) {
    for (int id : bp.groups[g]) {
      gis[g].push_back(inst[id]);
      gms[g].push_back(mus[id]);
    }
    gr.emplace_back(new GroupRun<T>());
    r = gr.back()->begin(bp.gplans[g], gis[g].data(), gms[g].data(), max_iter, o, w + bp.goff[g], s, nullptr,
                         nullptr, nullptr);
    if (r != FFCZ_OK) return r;
  }
  HIPCHK(hipStreamWaitEvent(s, g_streams.ready1d, 0));
  // one chunk of everything: the groups on a, the tiled 1D classes on b, forked from and joined into a
  auto enqueue_all = [&](hipStream_t a, hipStream_t b) -> hipError_t {
    hipError_t e = hipEventRecord(g_streams.cfork, a);
    if (e == hipSuccess) e = hipStreamWaitEvent(b, g_streams.cfork, 0);
    for (size_t g = 0; g < ng && e == hipSuccess; ++g) e = gr[g]->enqueue_chunk(a);
    if (e == hipSuccess) e = sr.enqueue_chunk(b);
    if (e == hipSuccess) e = hipEventRecord(g_streams.cjoin, b);
    if (e == hipSuccess) e = hipStreamWaitEvent(a, g_streams.cjoin, 0);
    return e;
  };
  hipGraphExec_t gexec = nullptr;
  if (o.use_graph && !g_prof.on) {
    GraphKey key{{-2}};
    for (size_t g = 0; g < ng; ++g) {
      const GraphKey gk = gr[g]->graph_key();
      key.k.insert(key.k.end(), gk.k.begin(), gk.k.end());
    }
    sr.key_into(key);
    std::lock_guard<std::mutex> lk(g_sig_graphs_m);
    gexec = sig_graphs().find(key);
    if (!gexec) {
      HIPCHK(hipStreamBeginCapture(g_streams.cap, hipStreamCaptureModeThreadLocal));
      const hipError_t ce = enqueue_all(g_streams.cap, g_streams.cap2);
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(g_streams.cap, &graph);
      if (ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(FFCZ_E_HIP, std::string("capture of the batch rounds: ") + hipGetErrorString(ce));
      }
      HIPCHK(ee);
      const hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(ie);
      sig_graphs().put(key, gexec);
    }
  }
  // host copies of every group's states and of the signal states, polled once per chunk
  size_t hbytes = sizeof(SigStats) * bp.sig_ids.size();
  std::vector<size_t> hoff(ng);
  for (size_t g = 0; g < ng; ++g) {
    hoff[g] = hbytes;
    hbytes += sizeof(DevState) * (size_t)bp.gplans[g].B;
  }
  HIPCHK(g_host_sigstate.reserve(hbytes));
  char* hb = (char*)g_host_sigstate.p;
  const int chunk = o.graph_chunk > 0 ? o.graph_chunk : 4;
  for (int enq = 0;; enq += chunk) {
    if (gexec) HIPCHK(hipGraphLaunch(gexec, s));
    else HIPCHK(enqueue_all(s, s1));
    HIPCHK(hipMemcpyAsync(hb, w + bp.off_sstats, sizeof(SigStats) * bp.sig_ids.size(), hipMemcpyDeviceToHost, s));
    for (size_t g = 0; g < ng; ++g)
      HIPCHK(hipMemcpyAsync(hb + hoff[g], gr[g]->c.st(), sizeof(DevState) * (size_t)bp.gplans[g].B,
                            hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool all = sr.all_done((const SigStats*)hb);
    for (size_t g = 0; g < ng && all; ++g) {
      const DevState* hs = (const DevState*)(hb + hoff[g]);
      for (int64_t b = 0; b < bp.gplans[g].B; ++b) all = all && hs[b].done;
    }
    if (all) break;
    if (enq > max_iter + 2 * chunk + 2) return fail(FFCZ_E_HIP, "batch did not report completion");
  }
  // the tiled classes' end on s1 (after the loop), the groups' ends on s
  HIPCHK(hipEventRecord(g_streams.looped, s));
  HIPCHK(hipStreamWaitEvent(s1, g_streams.looped, 0));
  r = sr.end();
  if (r != FFCZ_OK) return r;
  for (size_t g = 0; g < ng; ++g) {
    std::vector<int32_t> gs(gis[g].size(), FFCZ_OK);
    std::vector<ffcz_stats> gst(gis[g].size());
    r = gr[g]->end(gst.data(), gs.data());
    if (r != FFCZ_OK) return r;
    for (size_t k = 0; k < gis[g].size(); ++k) {
      status[bp.groups[g][k]] = gs[k];
      if (stats) stats[bp.groups[g][k]] = gst[k];
    }
  }
  return FFCZ_OK;
}

int32_t worst(const std::vector<int32_t>& st) {
  int32_t w = FFCZ_OK;
  for (int32_t v : st) {
    if (v < 0) return v;
    w = std::max(w, v);
  }
  return w;
}

// Checked arguments of a single-field call on the plan path.
struct SingleCall {
  Plan p;
  ffcz_options o;
  double mu = 0.0;
  ffcz_instance in;
};

int32_t single_setup(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, const void* xb, void* y,
                     double eps_s, double delta_f, int32_t max_iter, const ffcz_options* opts, SingleCall& sc) {
  int32_t r = make_plan(dtype, ndim, shape, max_iter, 1, sc.p);
  if (r != FFCZ_OK) return r;
  if (!x || !xb || !y) return fail(FFCZ_E_INVALID, "null data pointer");
  if (x == xb || x == y) return fail(FFCZ_E_INVALID, "x_orig must not alias x_base or x_out");
  if (!std::isfinite(eps_s) || eps_s < 0) return fail(FFCZ_E_INVALID, "eps_s must be finite and >= 0");
  if (!std::isfinite(delta_f) || delta_f < 0) return fail(FFCZ_E_INVALID, "delta_f must be finite and >= 0");
  if (((uintptr_t)x & 15) || ((uintptr_t)xb & 15) || ((uintptr_t)y & 15))
    return fail(FFCZ_E_WORKSPACE, "data pointers must be 16-byte aligned");
  if (opts) sc.o = *opts;
  else ffcz_default_options(&sc.o);
  if (sc.o.masks_out && sc.p.dt == FFCZ_F64 && col_block_cols(1, sc.p.Lx, 0) < 8)
    return fail(FFCZ_E_SHAPE, "mask recording needs at least 8 columns per block");
  // no margin given: FP64 takes 2^-16, FP32 derives mu from x on the device (no host round trip)
  sc.mu = sc.o.margin_rel > 0.0 ? sc.o.margin_rel : (dtype == FFCZ_F64 ? std::ldexp(1.0, -16) : 0.0);
  if (!(sc.mu < 1.0)) return fail(FFCZ_E_INVALID, "margin_rel must be in [0, 1)");
  memset(&sc.in, 0, sizeof(sc.in));
  sc.in.ndim = ndim;
  for (int i = 0; i < ndim; ++i) sc.in.shape[i] = shape[i];
  sc.in.x_orig = x;
  sc.in.x_base = xb;
  sc.in.x_out = y;
  sc.in.eps_s = eps_s;
  sc.in.delta_f = delta_f;
  return FFCZ_OK;
}

// host_state: null for the ordinary call; else the no-allocation form (see correct_group).
int32_t single_run(SingleCall& sc, char* ws, hipStream_t s, ffcz_stats* stats, DevState* host_state) {
  const double* mus = sc.mu > 0.0 ? &sc.mu : nullptr;
  int32_t status = FFCZ_OK;
  const int32_t r =
      sc.p.dt == FFCZ_F32
          ? correct_group<float>(sc.p, &sc.in, mus, sc.p.max_iter, sc.o, ws, s, stats, &status, host_state)
          : correct_group<double>(sc.p, &sc.in, mus, sc.p.max_iter, sc.o, ws, s, stats, &status, host_state);
  if (r != FFCZ_OK) return r;
  if (stats) stats->status = status;
  if (status == FFCZ_E_NONFINITE) return fail(FFCZ_E_NONFINITE, "x or x_hat holds NaN or Inf");
  if (status == FFCZ_VERIFY_FAILED) g_err = "FP64 re-verification failed";
  return status;
}

// CompactEdits + QuantizeEdits over one coordinate set: block counts, their scan, then
// flags and codes.  tot receives the number of codes.
template <typename T>
hipError_t code_set(const EditSet<T>& set, int64_t nb, unsigned long long* offs, unsigned long long* tot,
                    uint8_t* flags, int32_t* codes, double step, unsigned* status, hipStream_t s) {
  if (nb == 0) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, tot, (int64_t)1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(edit_count_kernel<T>, dim3((unsigned)nb), dim3(64 * kEditWaves), 0, s, set, offs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(edit_scan_kernel, dim3(1), dim3(1024), 0, s, offs, nb, tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(edit_write_kernel<T>, dim3((unsigned)nb), dim3(64 * kEditWaves), 0, s, set,
                     (const unsigned long long*)offs, flags, codes, step, status);
  return hipGetLastError();
}

// The inverse for the decoder: dense dequantised edits from flags and codes.
template <typename TO>
hipError_t expand_set(const EditSet<TO>& set, int64_t nb, unsigned long long* offs, unsigned long long* tot,
                      const uint8_t* flags, const int32_t* codes, int64_t ncodes, double step, unsigned* status,
                      hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(flag_count_kernel, dim3((unsigned)nb), dim3(64 * kEditWaves), 0, s, flags, set.ncoord, offs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(edit_scan_kernel, dim3(1), dim3(1024), 0, s, offs, nb, tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(edit_expand_kernel<TO>, dim3((unsigned)nb), dim3(64 * kEditWaves), 0, s, set, flags, codes,
                     ncodes, (const unsigned long long*)offs, step, (const unsigned long long*)tot, status);
  return hipGetLastError();
}

template <typename T>
EditSet<T> spatial_set(void* base, int64_t n) {
  EditSet<T> e;
  memset(&e, 0, sizeof(e));
  e.val = (T*)base;
  e.ncoord = n;
  return e;
}
template <typename T>
EditSet<T> freq_set(const Plan& p, void* spec) {
  EditSet<T> e;
  memset(&e, 0, sizeof(e));
  e.val = (T*)spec;
  e.ncoord = 2 * p.nrows * p.ncols;
  e.freq = 1;
  e.ncols = (int32_t)p.ncols;
  e.pitch = p.pitch;
  e.plane = p.plane;
  e.lg_rpp = p.lg_rpp;
  return e;
}

// Encoder after the loop: code both sets, export the accumulators when asked, and read
// back the code counts and the status word.
template <typename T>
int32_t code_edits(const Plan& p, const EditLayout& L, char* ws, void* sflags, int32_t* scodes, void* fflags,
                   int32_t* fcodes, double step_s, double step_f, void* sexp, void* fexp, hipStream_t s,
                   int64_t* nnz_s, int64_t* nnz_f) {
  unsigned long long* tot = (unsigned long long*)(ws + L.off_tot);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, tot, (int64_t)4);
  HIPCHK(hipGetLastError());
  unsigned* status = (unsigned*)(tot + 2);
  const EditSet<T> ss = spatial_set<T>(ws + L.off_S, L.ncs);
  const EditSet<T> fs = freq_set<T>(p, ws + L.off_F);
  HIPCHK(code_set<T>(ss, L.nbs, (unsigned long long*)(ws + L.off_offs), tot, (uint8_t*)sflags, scodes, step_s,
                     status, s));
  HIPCHK(code_set<T>(fs, L.nbf, (unsigned long long*)(ws + L.off_offf), tot + 1, (uint8_t*)fflags, fcodes, step_f,
                     status, s));
  if (sexp && L.ncs) {
    hipLaunchKernelGGL(edit_export_kernel<T>, dim3((unsigned)((L.ncs + 255) / 256)), dim3(256), 0, s, ss, (T*)sexp);
    HIPCHK(hipGetLastError());
  }
  if (fexp && L.ncf) {
    hipLaunchKernelGGL(edit_export_kernel<T>, dim3((unsigned)((L.ncf + 255) / 256)), dim3(256), 0, s, fs, (T*)fexp);
    HIPCHK(hipGetLastError());
  }
  unsigned long long h[3];
  HIPCHK(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *nnz_s = (int64_t)h[0];
  *nnz_f = (int64_t)h[1];
  if ((unsigned)h[2] & kEditCodeRange)
    return fail(FFCZ_E_INVALID, "an edit's code falls outside int32 (fewer code bits m, or a zero bound with edits)");
  return FFCZ_OK;
}

// Decoder: y = x_hat + s + IFFT(f) from flags and codes (Sec. IV-B, applying edits).
template <typename T>
int32_t decode_impl(const Plan& p, const EditLayout& L, char* ws, const void* xb, const void* sflags,
                    const int32_t* scodes, int64_t nnz_s, const void* fflags, const int32_t* fcodes, int64_t nnz_f,
                    double step_s, double step_f, void* y, hipStream_t s) {
  Ctx c{&p, ws, s};
  StateInit si;
  memset(&si, 0, sizeof(si));
  si.inv_n = 1.0 / (double)p.N;
  si.px = y;  // the expanded spatial edits, read back by the closing pass
  si.pxb = xb;
  si.py = y;
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, c.st(), (int64_t)1, (const StateInit*)nullptr, si,
                     c.viol(), (int64_t)1);
  HIPCHK(hipGetLastError());
  HIPCHK(write_twiddles(c));
  unsigned long long* tot = (unsigned long long*)(ws + L.off_tot);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, tot, (int64_t)4);
  HIPCHK(hipGetLastError());
  unsigned* status = (unsigned*)(tot + 2);
  // spatial edits straight into y (the field's dtype), frequency edits into Z
  HIPCHK(expand_set<T>(spatial_set<T>(y, L.ncs), L.nbs, (unsigned long long*)(ws + L.off_offs), tot,
                       (const uint8_t*)sflags, scodes, nnz_s, step_s, status, s));
  HIPCHK(expand_set<T>(freq_set<T>(p, c.Z()), L.nbf, (unsigned long long*)(ws + L.off_offf), tot + 1,
                       (const uint8_t*)fflags, fcodes, nnz_f, step_f, status, s));
  // inverse transforms: x, then y (3D), then the last-axis C2R with 1/N and the sum
  const char* twb = (const char*)c.twT();
  HIPCHK(run_col<T>(p.dt, COL_INV_NS, 0, geom_x(p, p.pitch, p.plane), p, c.Z(), c.Z(), twb + sizeof(cx<T>) * p.twx,
                    c.st(), nullptr, nullptr, s));
  if (p.nd == 3)
    HIPCHK(run_col<T>(p.dt, COL_INV_NS, 0, geom_y(p, p.pitch, p.plane), p, c.Z(), c.Z(),
                      twb + sizeof(cx<T>) * p.twy, c.st(), nullptr, nullptr, s));
  const hipError_t de = run_row<T, T>(p.dt, p.dt, ROW_DECODE, 0, p, p.pitch, p.plane, c.Z(), nullptr,
                                      twb + sizeof(cx<T>) * p.twz, c.st(), nullptr, nullptr, s);
  HIPCHK(de);
  unsigned long long h[3];
  HIPCHK(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if ((unsigned)h[2] & kEditFlagCount)
    return fail(FFCZ_E_INVALID, "the set flags and the code counts given disagree (spatial " +
                                    std::to_string(h[0]) + " vs " + std::to_string(nnz_s) + ", frequency " +
                                    std::to_string(h[1]) + " vs " + std::to_string(nnz_f) + ")");
  return FFCZ_OK;
}

// Pointwise spectral bound that keeps every shell of the power spectrum of x within rho:
// FP64 spectrum of x on the verification passes (their last-axis pass forms y - x; here y = x
// and x = a zero field), shell sums, shell bounds, then the bound of every entry.
template <typename T>
int32_t power_bounds_impl(const Plan& p, const BoundsLayout& L, char* ws, const void* x, double rho, int disk,
                          void* out, hipStream_t s) {
  Ctx c{&p, ws, s};
  StateInit si;
  memset(&si, 0, sizeof(si));
  si.inv_n = 1.0 / (double)p.N;
  si.px = ws + L.off_zero;
  si.py = const_cast<void*>(x);
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, c.st(), (int64_t)1, (const StateInit*)nullptr, si,
                     c.viol(), (int64_t)1);
  HIPCHK(hipGetLastError());
  const int64_t nz = (int64_t)p.N * (p.dt == FFCZ_F32 ? 4 : 8) / 8;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s,
                     (unsigned long long*)(ws + L.off_zero), nz);
  HIPCHK(hipGetLastError());
  HIPCHK(write_twiddles(c));
  const char* tb = (const char*)c.tw64();
  void* W = c.W();
  const hipError_t ez = run_row<double, T>(1, p.dt, ROW_VERIFY, kVerifyRowPlan, p, p.pitch64, p.plane64, nullptr, W,
                                           tb + 16 * p.twz8, c.st(), c.part(Ctx::PVZ), nullptr, s);
  HIPCHK(ez);
  if (p.nd == 3)
    HIPCHK(run_col<double>(1, COL_FWD_NS, 0, geom_y(p, p.pitch64, p.plane64), p, W, W, tb + 16 * p.twy, c.st(),
                           nullptr, nullptr, s));
  if (p.nd >= 2)
    HIPCHK(run_col<double>(1, COL_FWD_NS, 0, geom_x(p, p.pitch64, p.plane64), p, W, W, tb + 16 * p.twx, c.st(),
                           nullptr, nullptr, s));
  const SpecGeom g64{p.nrows, (int32_t)p.ncols, p.lg_rpp, p.pitch64, p.plane64};
  const int64_t n0 = p.nd >= 2 ? p.n[0] : 1, n1 = p.nd == 3 ? p.n[1] : 1, nl = p.n[p.nd - 1];
  double* part = (double*)(ws + L.off_shell);
  double* bins = (double*)(ws + L.off_bins);
  hipLaunchKernelGGL(shell_part_kernel, dim3((unsigned)L.nsb), dim3(256), 0, s, (const cx<double>*)W, g64, p.nd, n0,
                     n1, nl, L.nb, part);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(shell_bound_kernel, dim3((unsigned)((L.nb + 255) / 256)), dim3(256), 0, s,
                     (const double*)part, L.nsb, L.nb, rho, disk, bins);
  HIPCHK(hipGetLastError());
  const int64_t M = p.nrows * p.ncols;
  hipLaunchKernelGGL(shell_scatter_kernel<T>, dim3((unsigned)std::min<int64_t>(4096, (M + 255) / 256)), dim3(256), 0,
                     s, (const double*)bins, p.nrows, (int32_t)p.ncols, p.nd, n0, n1, (T*)out);
  HIPCHK(hipGetLastError());
  return FFCZ_OK;
}

// ---------------------------------------------------------------------------
// Huffman code construction (host side of LosslesslyCompressEdits).  The tree merges the two
// lightest nodes, ties going to the node created first (leaves in symbol order, then merged
// nodes in turn), so the code lengths depend on the frequency table alone; codes longer than
// kHuffMaxLen bits make every non-zero count (count + 1) / 2 and the tree is rebuilt.

constexpr int kHuffMaxLen = 32;
constexpr int64_t kHuffMaxAlpha = int64_t(1) << 24;

// The merges in O(n) after a sort: leaves sorted by (count, symbol), merged nodes appended to a
// second queue in creation order.  Merged weights never decrease, so both queues stay ordered
// by (weight, id) and the lighter front is the node a heap ordered by (weight, id) would pop
// (on equal weights the leaf, whose id is the smaller).
std::vector<uint8_t> huff_tree_lengths(const std::vector<unsigned long long>& c) {
  std::vector<uint8_t> len(c.size(), 0);
  std::vector<int64_t> present;
  std::vector<unsigned long long> w;  // leaf weights, leaf id = position in present
  for (size_t i = 0; i < c.size(); ++i)
    if (c[i]) {
      present.push_back((int64_t)i);
      w.push_back(c[i]);
    }
  const int64_t nl = (int64_t)present.size();
  if (nl == 0) return len;
  if (nl == 1) {
    len[present[0]] = 1;
    return len;
  }
  // sort the leaf ids by (weight, id): least significant digit radix sort on 11-bit digits
  // (stable, so equal weights keep id order)
  std::vector<int64_t> leaf(nl), tmp(nl);
  for (int64_t i = 0; i < nl; ++i) leaf[i] = i;
  unsigned long long wmax = 0;
  for (int64_t i = 0; i < nl; ++i) wmax = std::max(wmax, w[i]);
  for (int sh = 0; sh < 64 && (wmax >> sh) != 0; sh += 11) {
    std::vector<int64_t> bucket(2049, 0);
    for (int64_t i = 0; i < nl; ++i) bucket[((w[leaf[i]] >> sh) & 2047) + 1]++;
    for (int d = 0; d < 2048; ++d) bucket[d + 1] += bucket[d];
    for (int64_t i = 0; i < nl; ++i) tmp[bucket[(w[leaf[i]] >> sh) & 2047]++] = leaf[i];
    leaf.swap(tmp);
  }
  std::vector<unsigned long long> mw;  // merged weights, node id nl + k
  mw.reserve(nl - 1);
  std::vector<int64_t> parent(2 * nl - 1, -1);
  int64_t li = 0, mi = 0;
  auto pop = [&]() -> std::pair<unsigned long long, int64_t> {
    const bool take_leaf = li < nl && (mi >= (int64_t)mw.size() || w[leaf[li]] <= mw[mi]);
    if (take_leaf) {
      const int64_t id = leaf[li++];
      return {w[id], id};
    }
    const int64_t id = nl + mi;
    return {mw[mi++], id};
  };
  for (int64_t k = 0; k < nl - 1; ++k) {
    const auto a = pop();
    const auto b = pop();
    parent[a.second] = nl + k;
    parent[b.second] = nl + k;
    mw.push_back(a.first + b.first);
  }
  const int64_t nid = 2 * nl - 1;
  std::vector<int> depth(nid, 0);
  for (int64_t node = nid - 2; node >= 0; --node) depth[node] = depth[parent[node]] + 1;  // parents come later
  for (int64_t i = 0; i < nl; ++i) len[present[i]] = (uint8_t)std::min(depth[i], 255);
  return len;
}

std::vector<uint8_t> huff_lengths(std::vector<unsigned long long> c) {
  for (;;) {
    std::vector<uint8_t> len = huff_tree_lengths(c);
    int mx = 0;
    for (uint8_t l : len) mx = std::max<int>(mx, l);
    if (mx <= kHuffMaxLen) return len;
    for (auto& v : c)
      if (v) v = (v + 1) / 2;
  }
}

// Canonical tables: cnt[l] codes of length l, first[l] the first of them, idx[l] the position
// of the first in `sorted` (symbols ordered by length, then value), code[s] every symbol's code.
struct HuffTables {
  uint32_t first[kHuffMaxLen + 1], cnt[kHuffMaxLen + 1], idx[kHuffMaxLen + 1];
  std::vector<int32_t> sorted;
  std::vector<uint32_t> code;
};

HuffTables huff_tables(const std::vector<uint8_t>& len) {
  HuffTables t;
  memset(t.first, 0, sizeof(t.first));
  memset(t.cnt, 0, sizeof(t.cnt));
  memset(t.idx, 0, sizeof(t.idx));
  for (uint8_t l : len)
    if (l) t.cnt[l]++;
  uint64_t code = 0;
  uint32_t pos = 0;
  for (int l = 1; l <= kHuffMaxLen; ++l) {
    code = (code + (l > 1 ? t.cnt[l - 1] : 0)) << (l > 1 ? 1 : 0);
    t.first[l] = (uint32_t)code;
    t.idx[l] = pos;
    pos += t.cnt[l];
  }
  t.sorted.assign(pos, 0);
  t.code.assign(len.size(), 0);
  uint32_t fill[kHuffMaxLen + 1];
  for (int l = 0; l <= kHuffMaxLen; ++l) fill[l] = 0;
  for (size_t s = 0; s < len.size(); ++s) {
    const int l = len[s];
    if (!l) continue;
    t.sorted[t.idx[l] + fill[l]] = (int32_t)s;
    t.code[s] = t.first[l] + fill[l];
    fill[l]++;
  }
  return t;
}

// Stream layout in the caller's output buffer: the header, the code lengths (nalpha bytes,
// padded to 16), the chunk offsets (uint64), then the 32-bit words.
struct HuffHeader {
  uint32_t magic, width;
  int64_t nsym, lo, nalpha, nbits, nchunks, pad[2];
};
constexpr uint32_t kHuffMagic = 0x46554846u;  // "FHUF"

struct HuffLayout {
  size_t off_len, off_chunks, off_words, bytes;
};
HuffLayout huff_layout(int64_t n, int64_t nalpha, int64_t nbits) {
  HuffLayout L;
  L.off_len = sizeof(HuffHeader);
  L.off_chunks = align_up(L.off_len + (size_t)nalpha, 16);
  const int64_t nch = (n + kHuffChunk - 1) / kHuffChunk;
  L.off_words = align_up(L.off_chunks + 8 * (size_t)nch, 16);
  L.bytes = L.off_words + 4 * (size_t)((nbits + 31) / 32);
  return L;
}

// Workspace: minmax partials, the frequency table, lengths, codes, block offsets, totals and
// the decoder's tables.
struct HuffWs {
  size_t off_mm, off_counts, off_len, off_code, off_boff, off_tot, off_tab, off_sorted, bytes;
};
HuffWs huff_ws(int64_t n, int64_t nalpha) {
  HuffWs W;
  size_t off = 0;
  W.off_mm = off;
  off = align_up(off + 16 * 1024, 256);
  W.off_counts = off;
  off = align_up(off + 8 * (size_t)nalpha, 256);
  W.off_len = off;
  off = align_up(off + (size_t)nalpha, 256);
  W.off_code = off;
  off = align_up(off + 4 * (size_t)nalpha, 256);
  const int64_t nblk = (n + kHuffBlockSyms - 1) / kHuffBlockSyms;
  W.off_boff = off;
  off = align_up(off + 8 * (size_t)std::max<int64_t>(1, nblk), 256);
  W.off_tot = off;
  off = align_up(off + 64, 256);
  W.off_tab = off;
  off = align_up(off + 3 * 4 * (kHuffMaxLen + 1), 256);
  W.off_sorted = off;
  off = align_up(off + 4 * (size_t)nalpha, 256);
  W.bytes = off;
  return W;
}

// Scratch of ffcz_correct_noalloc (the array is declared at file scope, above): host
// code never passes the array's name to a kernel (on the host it names a host-side
// stand-in); it takes the device address hipGetSymbolAddress returns, once per device,
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_m;
char* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_on_current_device(char** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FFCZ_E_HIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_m);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255)) return fail(FFCZ_E_HIP, "scratch symbol address missing or misaligned");
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return FFCZ_OK;
}

}  // namespace

extern "C" {

int32_t ffcz_version(void) { return 100; }

const char* ffcz_last_error(void) { return g_err.c_str(); }

int32_t ffcz_set_tuning(int32_t mode, const char* cache_path) {
  if (mode < 0 || mode > 4) return fail(FFCZ_E_INVALID, "tuning mode must be 0 to 4");
  std::lock_guard<std::mutex> g(g_tuner.m);
  g_tuner.init_locked();
  g_tuner.mode = mode;
  if (cache_path) {
    g_tuner.path = cache_path;
    g_tuner.loaded = false;
    g_tuner.load_locked();
  }
  return FFCZ_OK;
}

void ffcz_clear_tuning(void) {
  std::lock_guard<std::mutex> g(g_tuner.m);
  g_tuner.tab.clear();
  g_tuner.loaded = true;
}

int32_t ffcz_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return FFCZ_OK;
  if (!dst || !src) return fail(FFCZ_E_INVALID, "null pointer");
  if (((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return fail(FFCZ_E_INVALID, "pointers must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 > 0) {
    for (int64_t v0 = 0; v0 < n16; v0 += (int64_t)1 << 36) {  // grid x holds 2^31 - 1 blocks
      const int64_t nv = std::min<int64_t>((int64_t)1 << 36, n16 - v0);
      hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, (uint4*)dst + v0,
                         (const uint4*)src + v0, nv);
      HIPCHK(hipGetLastError());
    }
  }
  const int tail = (int)(bytes - (size_t)n16 * 16);
  if (tail > 0) {
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(16), 0, s, (unsigned char*)dst + n16 * 16,
                       (const unsigned char*)src + n16 * 16, tail);
    HIPCHK(hipGetLastError());
  }
  return FFCZ_OK;
}

int32_t ffcz_copy_columns(void* dst, const void* src, int64_t n_axis, int64_t axis_stride, int64_t n_fixed,
                          int64_t fixed_stride, int64_t row_bytes, void* stream) {
  if (n_axis < 0 || n_fixed < 0 || row_bytes < 0 || axis_stride < 0 || fixed_stride < 0)
    return fail(FFCZ_E_INVALID, "negative count, stride or row size");
  if (n_axis == 0 || n_fixed == 0 || row_bytes == 0) return FFCZ_OK;
  if (!dst || !src) return fail(FFCZ_E_INVALID, "null pointer");
  if ((((uintptr_t)dst | (uintptr_t)src) & 15) || ((axis_stride | fixed_stride | row_bytes) & 15))
    return fail(FFCZ_E_INVALID, "pointers, strides and the row size must be multiples of 16 bytes");
  const int64_t tiles = (row_bytes + 127) / 128;
  if (tiles > INT32_MAX || n_fixed > INT32_MAX / tiles) return fail(FFCZ_E_INVALID, "too many tiles for one launch");
  hipLaunchKernelGGL(copy_columns_kernel, dim3((unsigned)(n_fixed * tiles)), dim3(256), 0, (hipStream_t)stream,
                     (char*)dst, (const char*)src, n_axis, axis_stride, fixed_stride, row_bytes, (int32_t)tiles);
  HIPCHK(hipGetLastError());
  return FFCZ_OK;
}

void ffcz_profile_enable(int32_t on) {
  g_prof.on = on != 0;
  for (int k = 0; k < PK_COUNT; ++k) {
    g_prof.ms[k] = 0.0;
    g_prof.cnt[k] = 0;
  }
}

void ffcz_profile_select(uint32_t kinds) { g_prof.kinds = kinds; }

int32_t ffcz_profile_read(ffcz_profile* out) {
  if (!out) return fail(FFCZ_E_INVALID, "null pointer");
  for (auto& ev : g_prof.pending) {
    if (ev.keep == 1) {
      float ms = 0.f;
      if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
        g_prof.ms[ev.kind] += ms;
        g_prof.cnt[ev.kind] += 1;
      }
    } else {
      (void)hipEventSynchronize(ev.b);
    }
    g_prof.pool.push_back(ev.a);
    g_prof.pool.push_back(ev.b);
  }
  g_prof.pending.clear();
  memset(out, 0, sizeof(*out));
  for (int k = 0; k < PK_COUNT && k < FFCZ_PROFILE_KINDS; ++k) {
    out->ms[k] = g_prof.ms[k];
    out->count[k] = g_prof.cnt[k];
    g_prof.ms[k] = 0.0;
    g_prof.cnt[k] = 0;
  }
  return FFCZ_OK;
}

void ffcz_default_options(ffcz_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->verify_fp64 = 1;
  o->graph_chunk = 4;
  o->use_graph = 1;
  o->resident_1d = 1;
  o->tiled_1d_lg = 0;
}

size_t ffcz_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter) {
  if (route_1d(ndim, shape)) {
    const ffcz_instance in = one_instance(ndim, shape, nullptr, nullptr, nullptr, 0.0, 0.0);
    return ffcz_batched_workspace_bytes(dtype, 1, &in, max_iter < 0 ? 0 : max_iter);
  }
  Plan p;
  std::string keep = g_err;
  if (make_plan(dtype, ndim, shape, max_iter < 0 ? 0 : max_iter, 1, p) != FFCZ_OK) return 0;
  g_err = keep;
  return p.bytes;
}

size_t ffcz_mask_bytes(int32_t ndim, const int64_t* shape, int32_t rounds) {
  if (route_1d(ndim, shape)) return 0;  // the 1D signal path records no masks
  Plan p;
  std::string keep = g_err;
  if (rounds < 0 || make_plan(FFCZ_F32, ndim, shape, rounds, 1, p) != FFCZ_OK) return 0;
  g_err = keep;
  return (size_t)(rounds + 1) * p.s_plane_bytes + (size_t)rounds * 2 * p.f_plane_bytes;
}

int32_t ffcz_suggest_margin(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, double delta_f,
                            void* ws, size_t ws_bytes, void* stream, double* mu_out) {
  int64_t N = 1;
  if (route_1d(ndim, shape)) {
    int64_t sq[3];
    const int nd = squeeze(ndim, shape, sq);
    if (nd == 1) N = sq[0];
    if (N > (int64_t)1 << 19) return fail(FFCZ_E_SHAPE, "1D lengths must be at most 2^19");
    if (dtype != FFCZ_F32 && dtype != FFCZ_F64) return fail(FFCZ_E_INVALID, "dtype must be FFCZ_F32 or FFCZ_F64");
  } else {
    Plan p;
    int32_t r = make_plan(dtype, ndim, shape, 0, 1, p);
    if (r != FFCZ_OK) return r;
    N = p.N;
  }
  if (!x || !mu_out) return fail(FFCZ_E_INVALID, "null pointer");
  if (!std::isfinite(delta_f) || delta_f < 0) return fail(FFCZ_E_INVALID, "delta_f must be finite and >= 0");
  if (dtype == FFCZ_F64) {
    *mu_out = std::ldexp(1.0, -16);
    return FFCZ_OK;
  }
  // the reduction's slots sit at the start of the workspace
  if (!ws || ws_bytes < sizeof(double) * (kUlpSlots + 1) || ((uintptr_t)ws & 255))
    return fail(FFCZ_E_WORKSPACE, "workspace too small or misaligned");
  hipStream_t s = (hipStream_t)stream;
  double* slots = (double*)ws;
  const int nsl = ulp_slots(N);
  const MarginJob job{(const float*)x, N, delta_f};
  hipLaunchKernelGGL(ulp_part_kernel, dim3((unsigned)nsl), dim3(256), 0, s, job, (const MarginJob*)nullptr, slots);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(margin_kernel, dim3(1), dim3(256), 0, s, (const double*)slots, job,
                     (const MarginJob*)nullptr, (int)FFCZ_F32, slots + kUlpSlots, (DevState*)nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(g_host_misc.reserve(sizeof(double)));
  HIPCHK(hipMemcpyAsync(g_host_misc.p, slots + kUlpSlots, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *mu_out = *(const double*)g_host_misc.p;
  return FFCZ_OK;
}

int32_t ffcz_correct(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, const void* xb, void* y,
                     double eps_s, double delta_f, int32_t max_iter, const ffcz_options* opts, void* ws,
                     size_t ws_bytes, void* stream, ffcz_stats* stats) {
  if (route_1d(ndim, shape)) {
    // one signal of any length on the 1D path, as a batch of one
    if (opts && (opts->masks_out || opts->viol_per_round))
      return fail(FFCZ_E_INVALID, "masks and per-check counts are recorded for power-of-two fields only");
    if (!x || !xb || !y) return fail(FFCZ_E_INVALID, "null data pointer");
    const ffcz_instance in = one_instance(ndim, shape, x, xb, y, eps_s, delta_f);
    ffcz_stats st;
    memset(&st, 0, sizeof(st));
    const int32_t r = ffcz_correct_batched(dtype, 1, &in, max_iter, opts, ws, ws_bytes, stream, &st);
    if (r == FFCZ_E_NONFINITE) g_err = "x or x_hat holds NaN or Inf";
    if (stats && st.status == r) *stats = st;
    return r;
  }
  SingleCall sc;
  int32_t r = single_setup(dtype, ndim, shape, x, xb, y, eps_s, delta_f, max_iter, opts, sc);
  if (r != FFCZ_OK) return r;
  if (!ws || ws_bytes < sc.p.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte and data 16-byte aligned");
  return single_run(sc, (char*)ws, (hipStream_t)stream, stats, nullptr);
}

int32_t ffcz_correct_noalloc(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, const void* xb,
                             void* y, double eps_s, double delta_f, int32_t max_iter, const ffcz_options* opts,
                             void* stream, ffcz_stats* stats) {
  if (route_1d(ndim, shape))
    return fail(FFCZ_E_SHAPE, "ffcz_correct_noalloc takes power-of-two fields only (the 1D signal path stages "
                              "its descriptors in pinned host memory)");
  SingleCall sc;
  int32_t r = single_setup(dtype, ndim, shape, x, xb, y, eps_s, delta_f, max_iter, opts, sc);
  if (r != FFCZ_OK) return r;
  if (sc.p.bytes > kScratchBytes)
    return fail(FFCZ_E_WORKSPACE, "ffcz_correct_noalloc: this shape and round cap need " +
                                      std::to_string(sc.p.bytes) + " bytes of scratch, above the fixed " +
                                      std::to_string(kScratchBytes) + " (FFCZ_NOALLOC_SCRATCH_BYTES)");
  char* ws = nullptr;
  r = scratch_on_current_device(&ws);
  if (r != FFCZ_OK) return r;
  DevState host_state;  // the loop state is read back into this (no pinned staging)
  return single_run(sc, ws, (hipStream_t)stream, stats, &host_state);
}

size_t ffcz_bounds_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter) {
  if (route_1d(ndim, shape)) return 0;
  Plan p;
  std::string keep = g_err;
  if (make_plan(dtype, ndim, shape, max_iter < 0 ? 0 : max_iter, 1, p) != FFCZ_OK) return 0;
  g_err = keep;
  return bounds_layout(p).bytes;
}

int32_t ffcz_correct_bounds(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, const void* xb,
                            void* y, double eps_s, double delta_f, const ffcz_bounds* bnd, int32_t max_iter,
                            const ffcz_options* opts, void* ws, size_t ws_bytes, void* stream, ffcz_stats* stats) {
  if (route_1d(ndim, shape))
    return fail(FFCZ_E_SHAPE, "pointwise bounds take fields that run on the multidimensional passes");
  SingleCall sc;
  int32_t r = single_setup(dtype, ndim, shape, x, xb, y, eps_s, delta_f, max_iter, opts, sc);
  if (r != FFCZ_OK) return r;
  if (sc.o.masks_out) return fail(FFCZ_E_INVALID, "masks are not recorded with pointwise bounds");
  ffcz_bounds b;
  memset(&b, 0, sizeof(b));
  if (bnd) b = *bnd;
  if (((uintptr_t)b.eps_s & 15) || ((uintptr_t)b.delta_re & 15) || ((uintptr_t)b.delta_im & 15))
    return fail(FFCZ_E_WORKSPACE, "bound arrays must be 16-byte aligned");
  const BoundsLayout L = bounds_layout(sc.p);
  if (!ws || ws_bytes < L.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_bounds_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte aligned");
  char* w = (char*)ws;
  BoundsCfg bc;
  bc.pE = b.eps_s;
  bc.disk = b.disk ? 1 : 0;
  bc.dre = b.delta_re;
  bc.dim = bc.disk ? b.delta_re : b.delta_im;  // the disk bounds the modulus by delta_re
  bc.sre = delta_f;
  bc.sim = delta_f;
  bc.pD = w + L.off_D;
  bc.minpart = (unsigned long long*)(w + L.off_min);
  bc.bad = (unsigned long long*)(w + L.off_bad);
  const double* mus = sc.mu > 0.0 && sc.o.margin_rel > 0.0 ? &sc.mu : nullptr;
  hipStream_t s = (hipStream_t)stream;
  int32_t status = FFCZ_OK;
  r = dtype == FFCZ_F32 ? correct_group<float>(sc.p, &sc.in, mus, max_iter, sc.o, w, s, stats, &status, nullptr,
                                               nullptr, &bc)
                        : correct_group<double>(sc.p, &sc.in, mus, max_iter, sc.o, w, s, stats, &status, nullptr,
                                                nullptr, &bc);
  if (r != FFCZ_OK) return r;
  if (stats) stats->status = status;
  if (status == FFCZ_E_NONFINITE) return fail(FFCZ_E_NONFINITE, "x or x_hat holds NaN or Inf");
  if (status == FFCZ_VERIFY_FAILED) g_err = "FP64 re-verification against the pointwise bounds failed";
  return status;
}

int32_t ffcz_power_spectrum_bounds(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, double rho,
                                   int32_t disk, void* delta_out, void* ws, size_t ws_bytes, void* stream) {
  if (route_1d(ndim, shape))
    return fail(FFCZ_E_SHAPE, "power-spectrum bounds take fields that run on the multidimensional passes");
  Plan p;
  int32_t r = make_plan(dtype, ndim, shape, 0, 1, p);
  if (r != FFCZ_OK) return r;
  if (!x || !delta_out) return fail(FFCZ_E_INVALID, "null pointer");
  if (!std::isfinite(rho) || rho < 0) return fail(FFCZ_E_INVALID, "rho must be finite and >= 0");
  if (((uintptr_t)x & 15) || ((uintptr_t)delta_out & 15)) return fail(FFCZ_E_WORKSPACE, "data must be 16-byte aligned");
  const BoundsLayout L = bounds_layout(p);
  if (L.nb > kMaxShells) return fail(FFCZ_E_SHAPE, "too many shells");
  if (!ws || ws_bytes < L.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_bounds_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  return dtype == FFCZ_F32 ? power_bounds_impl<float>(p, L, (char*)ws, x, rho, disk ? 1 : 0, delta_out, s)
                           : power_bounds_impl<double>(p, L, (char*)ws, x, rho, disk ? 1 : 0, delta_out, s);
}

size_t ffcz_huffman_workspace_bytes(int64_t nsym, int64_t nalpha) {
  if (nsym < 0 || nalpha < 0 || nalpha > kHuffMaxAlpha) return 0;
  return huff_ws(nsym, nalpha).bytes;
}

int32_t ffcz_huffman_plan(const void* sym, int64_t nsym, int32_t width, void* ws, size_t ws_bytes, void* stream,
                          ffcz_huffman_sizes* plan) {
  if (!plan || (nsym > 0 && !sym)) return fail(FFCZ_E_INVALID, "null pointer");
  if (width != 1 && width != 4) return fail(FFCZ_E_INVALID, "width must be 1 or 4");
  if (nsym < 0) return fail(FFCZ_E_INVALID, "nsym must be >= 0");
  memset(plan, 0, sizeof(*plan));
  plan->nsym = nsym;
  if (nsym > 0) {
    if (!ws || ws_bytes < huff_ws(nsym, 0).bytes || ((uintptr_t)ws & 255))
      return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_huffman_workspace_bytes(nsym, 0) or misaligned");
    hipStream_t s = (hipStream_t)stream;
    const int g = (int)std::min<int64_t>(1024, (nsym + kHuffBlock - 1) / kHuffBlock);
    long long* mm = (long long*)ws;
    hipLaunchKernelGGL(huff_minmax_kernel, dim3((unsigned)g), dim3(kHuffBlock), 0, s, sym, (int)width, nsym, mm);
    HIPCHK(hipGetLastError());
    std::vector<long long> h(2 * (size_t)g);
    HIPCHK(hipMemcpyAsync(h.data(), mm, sizeof(long long) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    long long lo = h[0], hi = h[1];
    for (int b = 1; b < g; ++b) {
      lo = std::min(lo, h[2 * b]);
      hi = std::max(hi, h[2 * b + 1]);
    }
    plan->lo = lo;
    plan->nalpha = hi - lo + 1;
    if (plan->nalpha > kHuffMaxAlpha) return fail(FFCZ_E_INVALID, "alphabet wider than 2^24 symbols");
  }
  plan->ws_bytes = huff_ws(nsym, plan->nalpha).bytes;
  plan->out_bytes = huff_layout(nsym, plan->nalpha, 32 * nsym).bytes;
  return FFCZ_OK;
}

int32_t ffcz_huffman_encode(const void* sym, int64_t nsym, int32_t width, const ffcz_huffman_sizes* plan, void* out,
                            size_t out_bytes, void* ws, size_t ws_bytes, void* stream, size_t* used_bytes) {
  if (!plan || !out || (nsym > 0 && !sym)) return fail(FFCZ_E_INVALID, "null pointer");
  if (width != 1 && width != 4) return fail(FFCZ_E_INVALID, "width must be 1 or 4");
  if (plan->nsym != nsym || plan->nalpha < 0 || plan->nalpha > kHuffMaxAlpha)
    return fail(FFCZ_E_INVALID, "plan does not match the stream");
  if ((uintptr_t)out & 15) return fail(FFCZ_E_WORKSPACE, "output must be 16-byte aligned");
  const int64_t nalpha = plan->nalpha, lo = plan->lo;
  const HuffWs W = huff_ws(nsym, nalpha);
  if (!ws || ws_bytes < W.bytes || ((uintptr_t)ws & 255))
    return fail(FFCZ_E_WORKSPACE, "workspace smaller than the plan's ws_bytes or misaligned");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  char* o = (char*)out;
  HuffHeader hd;
  memset(&hd, 0, sizeof(hd));
  hd.magic = kHuffMagic;
  hd.width = (uint32_t)width;
  hd.nsym = nsym;
  hd.lo = lo;
  hd.nalpha = nalpha;
  hd.nchunks = (nsym + kHuffChunk - 1) / kHuffChunk;
  std::vector<uint8_t> len;
  if (nsym > 0) {
    // the global frequency table, then the code on the host
    unsigned long long* counts = (unsigned long long*)(w + W.off_counts);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((nalpha + 255) / 256)), dim3(256), 0, s, counts, nalpha);
    HIPCHK(hipGetLastError());
    const int g = (int)std::min<int64_t>(1024, (nsym + kHuffBlock - 1) / kHuffBlock);
    hipLaunchKernelGGL(huff_hist_kernel, dim3((unsigned)g), dim3(kHuffBlock), 0, s, sym, (int)width, nsym,
                       (int64_t)lo, nalpha, counts);
    HIPCHK(hipGetLastError());
    // through pinned staging: the table out, the lengths and codes back (the copies in are
    // complete at the synchronisation that reads the bit count, before the buffer is reused)
    HIPCHK(g_host_misc.reserve(8 * (size_t)nalpha));
    unsigned long long* hcp = (unsigned long long*)g_host_misc.p;
    HIPCHK(hipMemcpyAsync(hcp, counts, 8 * (size_t)nalpha, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    len = huff_lengths(std::vector<unsigned long long>(hcp, hcp + nalpha));
    const HuffTables t = huff_tables(len);
    uint8_t* dlen = (uint8_t*)(w + W.off_len);
    uint32_t* dcode = (uint32_t*)(w + W.off_code);
    uint32_t* hcode = (uint32_t*)g_host_misc.p;
    uint8_t* hlen = (uint8_t*)(hcode + nalpha);
    memcpy(hcode, t.code.data(), 4 * (size_t)nalpha);
    memcpy(hlen, len.data(), (size_t)nalpha);
    HIPCHK(hipMemcpyAsync(dlen, hlen, (size_t)nalpha, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dcode, hcode, 4 * (size_t)nalpha, hipMemcpyHostToDevice, s));
    // bits per block, block offsets, the total
    const int64_t nblk = (nsym + kHuffBlockSyms - 1) / kHuffBlockSyms;
    unsigned long long* boff = (unsigned long long*)(w + W.off_boff);
    unsigned long long* tot = (unsigned long long*)(w + W.off_tot);
    hipLaunchKernelGGL(huff_bits_kernel, dim3((unsigned)nblk), dim3(kHuffBlock), 0, s, sym, (int)width, nsym,
                       (int64_t)lo, (const uint8_t*)dlen, boff);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(edit_scan_kernel, dim3(1), dim3(1024), 0, s, boff, nblk, tot);
    HIPCHK(hipGetLastError());
    unsigned long long nbits = 0;
    HIPCHK(hipMemcpyAsync(&nbits, tot, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    hd.nbits = (int64_t)nbits;
    const HuffLayout L = huff_layout(nsym, nalpha, hd.nbits);
    if (out_bytes < L.bytes) return fail(FFCZ_E_WORKSPACE, "output smaller than the stream (" + std::to_string(L.bytes) + " bytes)");
    const int64_t nwords = (hd.nbits + 31) / 32;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)(((nwords + 1) / 2 + 255) / 256)), dim3(256), 0, s,
                       (unsigned long long*)(o + L.off_words), (nwords + 1) / 2);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(huff_encode_kernel, dim3((unsigned)nblk), dim3(kHuffBlock), 0, s, sym, (int)width, nsym,
                       (int64_t)lo, (const uint8_t*)dlen, (const uint32_t*)dcode, (const unsigned long long*)boff,
                       (unsigned int*)(o + L.off_words), (unsigned long long*)(o + L.off_chunks));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(o + L.off_len, dlen, (size_t)nalpha, hipMemcpyDeviceToDevice, s));
  }
  const HuffLayout L = huff_layout(nsym, nalpha, hd.nbits);
  if (out_bytes < L.bytes) return fail(FFCZ_E_WORKSPACE, "output smaller than the stream");
  HIPCHK(hipMemcpyAsync(o, &hd, sizeof(hd), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (used_bytes) *used_bytes = L.bytes;
  return FFCZ_OK;
}

int32_t ffcz_huffman_decode(const void* in, size_t in_bytes, int32_t width, void* sym_out, int64_t capacity, void* ws,
                            size_t ws_bytes, void* stream, int64_t* nsym_out) {
  if (!in || in_bytes < sizeof(HuffHeader)) return fail(FFCZ_E_INVALID, "input too short");
  if ((uintptr_t)in & 15) return fail(FFCZ_E_WORKSPACE, "input must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  HuffHeader hd;
  HIPCHK(hipMemcpyAsync(&hd, in, sizeof(hd), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hd.magic != kHuffMagic || (hd.width != 1 && hd.width != 4) || hd.nsym < 0 || hd.nalpha < 0 ||
      hd.nalpha > kHuffMaxAlpha || hd.nbits < 0)
    return fail(FFCZ_E_INVALID, "not a stream written by ffcz_huffman_encode");
  if ((int32_t)hd.width != width) return fail(FFCZ_E_INVALID, "symbol width differs from the stream's");
  if (hd.nchunks != (hd.nsym + kHuffChunk - 1) / kHuffChunk)
    return fail(FFCZ_E_INVALID, "chunk count does not match the symbol count");
  const HuffLayout L = huff_layout(hd.nsym, hd.nalpha, hd.nbits);
  if (in_bytes < L.bytes) return fail(FFCZ_E_INVALID, "input shorter than its stream");
  if (hd.nsym > capacity || (hd.nsym > 0 && !sym_out)) return fail(FFCZ_E_INVALID, "output holds fewer symbols than the stream");
  if (nsym_out) *nsym_out = hd.nsym;
  if (hd.nsym == 0) return FFCZ_OK;
  const HuffWs W = huff_ws(hd.nsym, hd.nalpha);
  if (!ws || ws_bytes < W.bytes || ((uintptr_t)ws & 255))
    return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_huffman_workspace_bytes(nsym, nalpha) or misaligned");
  // through pinned staging: the lengths out, the decoder's tables back
  const size_t tab_bytes = 3 * sizeof(uint32_t) * (kHuffMaxLen + 1);
  HIPCHK(g_host_misc.reserve(std::max<size_t>((size_t)hd.nalpha, tab_bytes + 4 * (size_t)hd.nalpha)));
  const char* ib = (const char*)in;
  HIPCHK(hipMemcpyAsync(g_host_misc.p, ib + L.off_len, (size_t)hd.nalpha, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<uint8_t> len((const uint8_t*)g_host_misc.p, (const uint8_t*)g_host_misc.p + hd.nalpha);
  for (uint8_t l : len)
    if (l > kHuffMaxLen) return fail(FFCZ_E_INVALID, "code length above 32 in the stream");
  const HuffTables t = huff_tables(len);
  // a prefix code: at most 2^l codes of length l after the shorter ones (Kraft), so every
  // window the decoder meets maps into the table or is reported
  uint64_t kraft = 0;  // sum of 2^(32 - l) over the codes, at most 2^32
  for (int l = 1; l <= kHuffMaxLen; ++l) kraft += (uint64_t)t.cnt[l] << (kHuffMaxLen - l);
  if (kraft > (1ull << kHuffMaxLen)) return fail(FFCZ_E_INVALID, "code lengths break the Kraft inequality");
  char* w = (char*)ws;
  uint32_t* tab = (uint32_t*)(w + W.off_tab);
  uint32_t* htab = (uint32_t*)g_host_misc.p;  // first, cnt, idx, then the sorted symbols
  memcpy(htab, t.first, sizeof(t.first));
  memcpy(htab + (kHuffMaxLen + 1), t.cnt, sizeof(t.cnt));
  memcpy(htab + 2 * (kHuffMaxLen + 1), t.idx, sizeof(t.idx));
  HIPCHK(hipMemcpyAsync(tab, htab, tab_bytes, hipMemcpyHostToDevice, s));
  if (!t.sorted.empty()) {
    memcpy((char*)htab + tab_bytes, t.sorted.data(), 4 * t.sorted.size());
    HIPCHK(hipMemcpyAsync(w + W.off_sorted, (char*)htab + tab_bytes, 4 * t.sorted.size(), hipMemcpyHostToDevice, s));
  }
  unsigned int* bad = (unsigned int*)(w + W.off_tot);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, (unsigned long long*)bad, (int64_t)1);
  HIPCHK(hipGetLastError());
  const int64_t nch = hd.nchunks;
  hipLaunchKernelGGL(huff_decode_kernel, dim3((unsigned)((nch + kHuffDecBlock - 1) / kHuffDecBlock)),
                     dim3(kHuffDecBlock), 0, s,
                     (const unsigned int*)(ib + L.off_words), (int64_t)((hd.nbits + 31) / 32),
                     (const unsigned long long*)(ib + L.off_chunks), hd.nsym, (const uint32_t*)tab,
                     (const uint32_t*)(tab + (kHuffMaxLen + 1)), (const uint32_t*)(tab + 2 * (kHuffMaxLen + 1)),
                     (const int32_t*)(w + W.off_sorted), (int64_t)hd.lo, (int)width, sym_out, bad);
  HIPCHK(hipGetLastError());
  unsigned int hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hb) return fail(FFCZ_E_INVALID, "the stream holds a bit pattern that is no code");
  return FFCZ_OK;
}

size_t ffcz_encode_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter) {
  if (route_1d(ndim, shape)) return 0;
  Plan p;
  std::string keep = g_err;
  if (make_plan(dtype, ndim, shape, max_iter < 0 ? 0 : max_iter, 1, p) != FFCZ_OK) return 0;
  g_err = keep;
  return edit_layout(p).bytes;
}

void ffcz_default_encode_options(ffcz_encode_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->m = 16;
  o->safety = 4.0;
}

int32_t ffcz_encode(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, const void* xb, double eps_s,
                    double delta_f, int32_t max_iter, const ffcz_options* opts, const ffcz_encode_options* eopts,
                    void* spat_flags, int32_t* spat_codes, void* freq_flags, int32_t* freq_codes, void* ws,
                    size_t ws_bytes, void* stream, ffcz_encode_stats* est) {
  if (route_1d(ndim, shape))
    return fail(FFCZ_E_SHAPE, "the encoder takes fields that run on the multidimensional passes (power-of-two extents)");
  ffcz_encode_options eo;
  if (eopts) eo = *eopts;
  else ffcz_default_encode_options(&eo);
  const int m = eo.m > 0 ? eo.m : 16;
  const double safety = eo.safety > 0.0 ? eo.safety : 4.0;
  if (m > 30) return fail(FFCZ_E_INVALID, "code length m must be at most 30");
  if (!std::isfinite(safety)) return fail(FFCZ_E_INVALID, "safety must be finite");
  if (!(eo.mu_s >= 0.0 && eo.mu_s < 0.5) || !(eo.mu_f >= 0.0 && eo.mu_f < 0.25))
    return fail(FFCZ_E_INVALID, "mu_s must lie in [0, 1/2) and mu_f in [0, 1/4)");
  if ((eo.mu_s > 0.0) != (eo.mu_f > 0.0)) return fail(FFCZ_E_INVALID, "give both shrinks or neither");
  SingleCall sc;
  // without y_out the closing pass does not run and nothing is written to the output pointer
  void* y = eo.y_out ? eo.y_out : const_cast<void*>(xb);
  int32_t r = single_setup(dtype, ndim, shape, x, xb, y, eps_s, delta_f, max_iter, opts, sc);
  if (r != FFCZ_OK) return r;
  if (!spat_flags || !spat_codes || !freq_flags || !freq_codes) return fail(FFCZ_E_INVALID, "null flag or code buffer");
  if (((uintptr_t)spat_flags & 15) || ((uintptr_t)spat_codes & 15) || ((uintptr_t)freq_flags & 15) ||
      ((uintptr_t)freq_codes & 15) || ((uintptr_t)eo.spat_edits_out & 15) || ((uintptr_t)eo.freq_edits_out & 15))
    return fail(FFCZ_E_WORKSPACE, "flag, code and edit buffers must be 16-byte aligned");
  const EditLayout L = edit_layout(sc.p);
  if (!ws || ws_bytes < L.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_encode_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (!eo.y_out) sc.o.verify_fp64 = 0;
  char* w = (char*)ws;
  EditCfg ed;
  ed.sacc = w + L.off_S;
  ed.facc = w + L.off_F;
  ed.derive = eo.mu_s == 0.0;
  ed.q = safety * std::ldexp(1.0, -m);
  ed.mu_s = eo.mu_s;
  ed.mu_f = eo.mu_f;
  ed.want_y = eo.y_out != nullptr;
  ed.amax = (unsigned long long*)(w + L.off_amax);
  double mu_s_used = 0.0;
  ed.mu_s_out = &mu_s_used;
  sc.mu = 0.5;  // placeholder: the encoder's own shrinks replace the margin (on the host or the device)
  hipStream_t s = (hipStream_t)stream;
  ffcz_stats lst;
  memset(&lst, 0, sizeof(lst));
  int32_t status = FFCZ_OK;
  const double* mus = &sc.mu;
  r = dtype == FFCZ_F32 ? correct_group<float>(sc.p, &sc.in, mus, max_iter, sc.o, w, s, &lst, &status, nullptr, &ed)
                        : correct_group<double>(sc.p, &sc.in, mus, max_iter, sc.o, w, s, &lst, &status, nullptr, &ed);
  if (r != FFCZ_OK) return r;
  lst.status = status;
  if (status == FFCZ_E_NONFINITE) return fail(FFCZ_E_NONFINITE, "x or x_hat holds NaN or Inf");
  const double step_s = std::ldexp(2.0 * eps_s, -m), step_f = std::ldexp(2.0 * delta_f, -m);
  int64_t nnz_s = 0, nnz_f = 0;
  r = dtype == FFCZ_F32 ? code_edits<float>(sc.p, L, w, spat_flags, spat_codes, freq_flags, freq_codes, step_s,
                                            step_f, eo.spat_edits_out, eo.freq_edits_out, s, &nnz_s, &nnz_f)
                        : code_edits<double>(sc.p, L, w, spat_flags, spat_codes, freq_flags, freq_codes, step_s,
                                             step_f, eo.spat_edits_out, eo.freq_edits_out, s, &nnz_s, &nnz_f);
  if (r != FFCZ_OK) return r;
  if (est) {
    memset(est, 0, sizeof(*est));
    est->loop = lst;
    est->nnz_s = nnz_s;
    est->nnz_f = nnz_f;
    est->step_s = step_s;
    est->step_f = step_f;
    // the shrinks in use: the state read back by the loop
    est->mu_f = lst.margin_used;
    est->mu_s = mu_s_used;
    est->m = m;
    est->status = status;
  }
  if (status == FFCZ_VERIFY_FAILED) g_err = "FP64 re-verification of y failed";
  return status;
}

int32_t ffcz_decode(int32_t dtype, int32_t ndim, const int64_t* shape, const void* xb, const void* spat_flags,
                    const int32_t* spat_codes, int64_t nnz_s, const void* freq_flags, const int32_t* freq_codes,
                    int64_t nnz_f, double step_s, double step_f, void* y, void* ws, size_t ws_bytes, void* stream) {
  if (route_1d(ndim, shape))
    return fail(FFCZ_E_SHAPE, "the decoder takes fields that run on the multidimensional passes (power-of-two extents)");
  Plan p;
  int32_t r = make_plan(dtype, ndim, shape, 0, 1, p);
  if (r != FFCZ_OK) return r;
  const EditLayout L = edit_layout(p);
  if (!xb || !y || !spat_flags || !freq_flags) return fail(FFCZ_E_INVALID, "null pointer");
  if ((nnz_s > 0 && !spat_codes) || (nnz_f > 0 && !freq_codes)) return fail(FFCZ_E_INVALID, "null code buffer");
  if (nnz_s < 0 || nnz_f < 0 || nnz_s > L.ncs || nnz_f > L.ncf) return fail(FFCZ_E_INVALID, "code counts out of range");
  if (xb == y) return fail(FFCZ_E_INVALID, "x_base and y must not alias");
  if (!std::isfinite(step_s) || !std::isfinite(step_f) || step_s < 0 || step_f < 0)
    return fail(FFCZ_E_INVALID, "steps must be finite and >= 0");
  if (((uintptr_t)xb & 15) || ((uintptr_t)y & 15) || ((uintptr_t)spat_flags & 15) || ((uintptr_t)freq_flags & 15) ||
      ((uintptr_t)spat_codes & 15) || ((uintptr_t)freq_codes & 15))
    return fail(FFCZ_E_WORKSPACE, "data, flag and code buffers must be 16-byte aligned");
  if (!ws || ws_bytes < L.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_encode_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  return dtype == FFCZ_F32 ? decode_impl<float>(p, L, (char*)ws, xb, spat_flags, spat_codes, nnz_s, freq_flags,
                                                freq_codes, nnz_f, step_s, step_f, y, s)
                           : decode_impl<double>(p, L, (char*)ws, xb, spat_flags, spat_codes, nnz_s, freq_flags,
                                                 freq_codes, nnz_f, step_s, step_f, y, s);
}

size_t ffcz_batched_workspace_bytes(int32_t dtype, int32_t count, const ffcz_instance* inst, int32_t max_iter) {
  BatchPlan bp;
  std::string keep = g_err;
  if (max_iter < 0 || batch_plan(dtype, count, inst, max_iter, bp) != FFCZ_OK) return 0;
  g_err = keep;
  return bp.bytes;
}

int32_t ffcz_correct_batched(int32_t dtype, int32_t count, const ffcz_instance* inst, int32_t max_iter,
                             const ffcz_options* opts, void* ws, size_t ws_bytes, void* stream, ffcz_stats* stats) {
  if (max_iter < 0) return fail(FFCZ_E_INVALID, "max_iter must be >= 0");
  BatchPlan bp;
  int32_t r = batch_plan(dtype, count, inst, max_iter, bp);
  if (r != FFCZ_OK) return r;
  if (!ws || ws_bytes < bp.bytes || ((uintptr_t)ws & 255))
    return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_batched_workspace_bytes() or misaligned");
  ffcz_options o;
  if (opts) o = *opts;
  else ffcz_default_options(&o);
  o.masks_out = nullptr;
  o.viol_per_round = nullptr;
  for (int i = 0; i < count; ++i) {
    const ffcz_instance& in = inst[i];
    if (!in.x_orig || !in.x_base || !in.x_out) return fail(FFCZ_E_INVALID, "null data pointer");
    if (in.x_orig == in.x_base || in.x_orig == in.x_out) return fail(FFCZ_E_INVALID, "x_orig must not alias");
    if (!std::isfinite(in.eps_s) || in.eps_s < 0 || !std::isfinite(in.delta_f) || in.delta_f < 0)
      return fail(FFCZ_E_INVALID, "bounds must be finite and >= 0");
    if (((uintptr_t)in.x_orig & 15) || ((uintptr_t)in.x_base & 15) || ((uintptr_t)in.x_out & 15))
      return fail(FFCZ_E_WORKSPACE, "data must be 16-byte aligned");
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  // margins: per instance (FP32: suggested from x, all members in one launch; FP64: 2^-16)
  std::vector<double> mus(count, o.margin_rel);
  if (!(o.margin_rel > 0.0) && count > 0) {
    std::vector<int64_t> Ns(count);
    for (int i = 0; i < count; ++i) {
      int64_t sq[3];
      const int nd = squeeze(inst[i].ndim, inst[i].shape, sq);
      int64_t N = 1;
      for (int d = 0; d < nd; ++d) N *= sq[d];
      Ns[i] = N;
    }
    if (dtype == FFCZ_F64) {
      for (int i = 0; i < count; ++i) mus[i] = std::ldexp(1.0, -16);
    } else {
      HIPCHK(g_host_misc.reserve(sizeof(MarginJob) * count + sizeof(double) * count));
      MarginJob* hj = (MarginJob*)g_host_misc.p;
      double* hmu = (double*)(hj + count);
      int64_t nmax = 1;
      for (int i = 0; i < count; ++i) {
        hj[i] = MarginJob{(const float*)inst[i].x_orig, Ns[i], inst[i].delta_f};
        nmax = std::max(nmax, Ns[i]);
      }
      MarginJob* dj = (MarginJob*)(w + bp.off_mjobs);
      double* dpart = (double*)(w + bp.off_msum);
      double* dmu = dpart + (size_t)count * kUlpSlots;
      HIPCHK(hipMemcpyAsync(dj, hj, sizeof(MarginJob) * count, hipMemcpyHostToDevice, s));
      const unsigned bx = (unsigned)ulp_slots(nmax);
      for (int c0 = 0; c0 < count; c0 += 65535) {  // grid y holds at most 65535 fields
        const int nc = std::min(65535, count - c0);
        hipLaunchKernelGGL(ulp_part_kernel, dim3(bx, (unsigned)nc), dim3(256), 0, s, MarginJob{},
                           (const MarginJob*)dj + c0, dpart + (size_t)c0 * kUlpSlots);
        HIPCHK(hipGetLastError());
      }
      hipLaunchKernelGGL(margin_kernel, dim3((unsigned)count), dim3(256), 0, s, (const double*)dpart, MarginJob{},
                         (const MarginJob*)dj, (int)FFCZ_F32, dmu, (DevState*)nullptr);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hmu, dmu, sizeof(double) * count, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < count; ++i) mus[i] = hmu[i];
    }
  }
  std::vector<int32_t> status(count, FFCZ_OK);
  if (!bp.sig_ids.empty() && !bp.groups.empty()) {
    r = dtype == FFCZ_F32 ? mixed_batch<float>(bp, inst, mus, max_iter, o, w, s, stats, status)
                          : mixed_batch<double>(bp, inst, mus, max_iter, o, w, s, stats, status);
    if (r != FFCZ_OK) return r;
  } else {
    r = pretune_sigs(bp, inst, mus.data(), o, w, s, g_host_sig);
    if (r != FFCZ_OK) return r;
    r = run_sigs(bp, inst, mus.data(), max_iter, o, w, s, g_host_sig, g_host_sigstate);
    if (r != FFCZ_OK) return r;
    for (size_t g = 0; g < bp.groups.size(); ++g) {
      const Plan& p = bp.gplans[g];
      std::vector<ffcz_instance> gi;
      std::vector<double> gm;
      for (int id : bp.groups[g]) {
        gi.push_back(inst[id]);
        gm.push_back(mus[id]);
      }
      std::vector<int32_t> gs(gi.size(), FFCZ_OK);
      std::vector<ffcz_stats> gst(gi.size());
      r = dtype == FFCZ_F32
              ? correct_group<float>(p, gi.data(), gm.data(), max_iter, o, w + bp.goff[g], s, gst.data(), gs.data())
              : correct_group<double>(p, gi.data(), gm.data(), max_iter, o, w + bp.goff[g], s, gst.data(), gs.data());
      if (r != FFCZ_OK) return r;
      for (size_t k = 0; k < gi.size(); ++k) {
        status[bp.groups[g][k]] = gs[k];
        if (stats) stats[bp.groups[g][k]] = gst[k];
      }
    }
  }
  r = collect_sigs(bp, inst, mus.data(), o, w, s, stats, status.data());
  if (r != FFCZ_OK) return r;
  if (stats)
    for (int i = 0; i < count; ++i) stats[i].status = status[i];
  const int32_t wst = worst(status);
  if (wst == FFCZ_VERIFY_FAILED) g_err = "FP64 re-verification failed for at least one instance";
  return wst;
}

int32_t ffcz_correct_backward(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t rounds, const void* masks,
                              const void* gy, void* gb, void* ws, size_t ws_bytes, void* stream) {
  if (route_1d(ndim, shape)) return fail(FFCZ_E_SHAPE, "the adjoint needs a power-of-two field (masks are recorded there)");
  Plan p;
  int32_t r = make_plan(dtype, ndim, shape, rounds, 1, p);
  if (r != FFCZ_OK) return r;
  if (!masks || !gy || !gb) return fail(FFCZ_E_INVALID, "null pointer");
  if (((uintptr_t)gy & 15) || ((uintptr_t)gb & 15)) return fail(FFCZ_E_WORKSPACE, "gradients must be 16-byte aligned");
  if (!ws || ws_bytes < p.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  // the last-axis plan the table holds for this geometry (no timing here): the adjoint's
  // last-axis passes take the direct form where the forward loop pass does
  if (p.H >= 64) {
    int vz = 0;
    r = tune_pass(tune_key_z(p), s, false, 0.98f, kRowVariants, [](int) { return hipSuccess; }, &vz);
    if (r != FFCZ_OK) return r;
    set_variants(p, 0, 0, vz);
  }
  if (dtype == FFCZ_F32) return backward_impl<float>(p, rounds, masks, gy, gb, ws, s);
  return backward_impl<double>(p, rounds, masks, gy, gb, ws, s);
}

}  // extern "C"
