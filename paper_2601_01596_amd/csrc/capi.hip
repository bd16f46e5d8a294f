// C ABI and host driver of the correction (declarations and contracts in ffcz.h).
//
// Per projection round the device runs, for a 3D field n0 x n1 x n2 with
// half-spectrum rows of H+1 = n2/2+1 entries:
//   y-fwd   Z -> A   C2C along axis 1
//   x-pass  A -> A   C2C along axis 0, count violations, clip Re/Im, inverse C2C
//   y-inv   A -> A   inverse C2C along axis 1
//   z-pass  A -> Z   C2R along axis 2, 1/N, clip eps, R2C
// (2D: x-pass Z -> A and z-pass A -> Z; 1D: the x-pass has length 1.)
// Z therefore always holds the spectrum of the last iterate eps_k while the
// check of round k runs, so when that check passes the output is the C2R of Z.
// The last block of every x-pass decides, on the device, whether the loop
// stops; every loop kernel returns at entry once the done-flag is set, so the
// host enqueues rounds in chunks and polls the flag once per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ffcz.h"
#include "common.hpp"
#include "launch.hpp"

namespace ffcz {
hipError_t launch_col_f32(int mode, int L, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_col_f64(int mode, int L, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_row_f32(int mode, int H, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_row_f64(int mode, int H, const void* args, int64_t nb, hipStream_t s);
hipError_t launch_row_verify_f32io(int H, const void* args, int64_t nb, hipStream_t s);

int col_block_cols(int dtype, int L) { return dtype == 0 ? pick_C<float>(L) : pick_C<double>(L); }
int row_block_rows(int H) { return pick_rows(H); }

hipError_t launch_col(int dtype, int mode, int L, const void* args, int64_t nb, hipStream_t s) {
  return dtype == 0 ? launch_col_f32(mode, L, args, nb, s) : launch_col_f64(mode, L, args, nb, s);
}
}  // namespace ffcz

using namespace ffcz;

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
  if (!g_prof.on) return launch();
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

struct Plan {
  int dt = 0;        // 0 f32, 1 f64
  int nd = 0;        // squeezed ndim
  int64_t n[3] = {1, 1, 1};
  int64_t N = 1;
  int H = 0;         // n_last / 2
  int64_t ncols = 0; // H + 1
  int64_t pitch = 0; // complex entries per spectrum row (working type)
  int64_t pitch64 = 0;
  int64_t nrows = 0; // N / n_last
  int Lx = 1, Ly = 0;
  int Ez = 1, Ey = 1, Ex = 1;
  // twiddle tables (complex entries): working type and double
  int64_t twz = 0, twy = 0, twx = 0, twT = 0;
  int64_t tw64z = 0, tw64y = 0, tw64x = 0, tw64 = 0;
  // blocks of each pass (one partial slot per block)
  int64_t nbz = 0, nbx = 0, nbvx = 0, pmax = 0;
  // workspace byte offsets
  size_t off_state = 0, off_viol = 0, off_part = 0, off_twT = 0, off_tw64 = 0, off_Z = 0, off_A = 0, bytes = 0;
  int32_t max_iter = 0;
  // masks
  int64_t s_row_w32 = 0, s_plane_bytes = 0, f_row_bytes = 0, f_plane_bytes = 0;
};

int pick_E_host(int L) { return pick_E(L); }

// Squeeze unit extents and check the supported shape set.
int32_t make_plan(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter, Plan& p) {
  if (dtype != FFCZ_F32 && dtype != FFCZ_F64) return fail(FFCZ_E_INVALID, "dtype must be FFCZ_F32 or FFCZ_F64");
  if (ndim < 1 || ndim > 3 || shape == nullptr) return fail(FFCZ_E_SHAPE, "ndim must be 1..3");
  if (max_iter < 0) return fail(FFCZ_E_INVALID, "max_iter must be >= 0");
  p = Plan();
  p.dt = dtype;
  p.max_iter = max_iter;
  int64_t sq[3];
  int nd = 0;
  for (int i = 0; i < ndim; ++i) {
    if (shape[i] < 1) return fail(FFCZ_E_SHAPE, "every extent must be >= 1");
    if (shape[i] > 1) sq[nd++] = shape[i];
  }
  if (nd == 0) return fail(FFCZ_E_SHAPE, "a single-point field is not supported (last extent must be >= 2)");
  const int64_t maxo = dtype == FFCZ_F32 ? 2048 : 1024;
  for (int i = 0; i < nd; ++i) {
    if (!is_pow2(sq[i])) return fail(FFCZ_E_SHAPE, "extents must be powers of two");
    if (i < nd - 1 && sq[i] > maxo) return fail(FFCZ_E_SHAPE, "leading extents above the supported maximum");
  }
  const int64_t nl = sq[nd - 1];
  if (nl < 2 || nl > kMaxLast) return fail(FFCZ_E_SHAPE, "last extent must be in [2, 4096]");
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
  if (nd == 1) {
    p.Lx = 1;
    p.Ly = 0;
  } else if (nd == 2) {
    p.Lx = (int)sq[0];
    p.Ly = 0;
  } else {
    p.Lx = (int)sq[0];
    p.Ly = (int)sq[1];
  }
  p.Ez = pick_E_host(p.H);
  p.Ex = pick_E_host(p.Lx);
  p.Ey = p.Ly ? pick_E_host(p.Ly) : 1;
  // twiddle layout: z (stages + H R2C twiddles), y stages, x stages
  p.twz = 0;
  p.twy = p.twz + host_twsize(p.H, p.Ez) + p.H;
  p.twx = p.twy + (p.Ly ? host_twsize(p.Ly, p.Ey) : 0);
  p.twT = p.twx + host_twsize(p.Lx, p.Ex) + 1;
  p.tw64z = p.twz;
  p.tw64y = p.twy;
  p.tw64x = p.twx;
  p.tw64 = p.twT;
  const size_t cs = dtype == FFCZ_F32 ? 8 : 16;
  {
    const int64_t outer_x = nd == 3 ? p.n[1] : 1;
    const int Cx = col_block_cols(dtype, p.Lx), Cx64 = col_block_cols(1, p.Lx);
    p.nbz = (p.nrows + row_block_rows(p.H) - 1) / row_block_rows(p.H);
    p.nbx = outer_x * ((p.ncols + Cx - 1) / Cx);
    p.nbvx = outer_x * ((p.ncols + Cx64 - 1) / Cx64);
    p.pmax = std::max(p.nbz, std::max(p.nbx, p.nbvx));
  }
  size_t off = 0;
  p.off_state = off;
  off = align_up(off + sizeof(DevState), 256);
  p.off_viol = off;
  off = align_up(off + sizeof(unsigned long long) * ((size_t)max_iter + 2), 256);
  // partial slots: x-pass counts | z-pass counts | verify-z max | verify-x count, max
  p.off_part = off;
  off = align_up(off + sizeof(unsigned long long) * 5 * (size_t)p.pmax, 256);
  p.off_twT = off;
  off = align_up(off + cs * (size_t)p.twT, 256);
  p.off_tw64 = off;
  off = align_up(off + 16 * (size_t)p.tw64, 256);
  p.off_Z = off;
  const size_t spec = cs * (size_t)p.nrows * (size_t)p.pitch;
  off = align_up(off + spec, 256);
  p.off_A = off;
  off = align_up(off + spec, 256);
  // the FP64 verification reuses Z..A (contiguous) as an FP64 spectrum
  const size_t spec64 = 16 * (size_t)p.nrows * (size_t)p.pitch64;
  if (p.off_Z + spec64 > off) off = align_up(p.off_Z + spec64, 256);
  p.bytes = off;
  // masks
  const int64_t sw64 = (nl + 63) / 64;
  const int64_t fw64 = (p.ncols + 63) / 64;
  p.s_row_w32 = 2 * sw64;
  p.s_plane_bytes = p.nrows * sw64 * 8;
  p.f_row_bytes = fw64 * 8;
  p.f_plane_bytes = p.nrows * fw64 * 8;
  return FFCZ_OK;
}

// ---------------------------------------------------------------------------
// set-up kernels

struct TwJob {
  int64_t off;  // complex entries from the table base
  int L, E, rtw;
};
struct TwJobs {
  TwJob j[3];
  int n;
  int dbl;  // 1: double table
};

__global__ void twiddle_kernel(void* base, TwJobs jobs) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t acc = 0;
  for (int jj = 0; jj < jobs.n; ++jj) {
    const TwJob& jb = jobs.j[jj];
    StageDesc d[32];
    const int ns = host_stages(jb.L, jb.E, d);
    int tsz = 0;
    for (int s = 0; s < ns; ++s)
      if (d[s].ns > 1) tsz += d[s].ns * (d[s].radix - 1);
    const int64_t cnt = tsz + (jb.rtw ? jb.L : 0);
    if (gid < acc + cnt) {
      const int64_t e = gid - acc;
      double num, den;  // angle = -2 pi num / den
      if (e < tsz) {
        int s = 0;
        for (; s < ns; ++s) {
          if (d[s].ns > 1 && e >= d[s].off && e < d[s].off + d[s].ns * (d[s].radix - 1)) break;
        }
        const int64_t loc = e - d[s].off;
        const int64_t m = loc / (d[s].radix - 1);
        const int64_t r = loc % (d[s].radix - 1) + 1;
        num = (double)(m * r);
        den = (double)d[s].ns * d[s].radix;
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

struct StateInit {
  double E, Ep, Delta, Dp, inv_n;
  int32_t max_iter, fixed, record_masks;
};

__global__ void state_init_kernel(DevState* st, unsigned long long* viol, int32_t nviol, StateInit p) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    DevState s;
    memset(&s, 0, sizeof(s));
    s.E = p.E;
    s.Ep = p.Ep;
    s.Delta = p.Delta;
    s.Dp = p.Dp;
    s.inv_n = p.inv_n;
    s.max_iter = p.max_iter;
    s.fixed = p.fixed;
    s.record_masks = p.record_masks;
    *st = s;
  }
  for (int i = t; i < nviol; i += gridDim.x * blockDim.x) viol[i] = 0ull;
}

template <typename T>
__global__ void ulp_kernel(const T* x, int64_t n, DevState* st) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float a = fabsf((float)x[i]);
    const double u = (double)nextafterf(a, INFINITY) - (double)a;
    s += u * u;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) b += red[w];
    atomicAdd(&st->ulp2_sum, b);
  }
}

// Per-round control: sum the x-pass partials into v_k, fold the spatial-clip
// partials of the z-pass that produced the checked iterate into the totals,
// and decide on the device whether the loop stops (Alg. 1: stop when no
// coefficient violates; also at the round cap, or on non-finite input).
__global__ void __launch_bounds__(1024) ctl_kernel(DevState* st, unsigned long long* viol,
                                                   const unsigned long long* xpart, int64_t nbx,
                                                   const unsigned long long* zpart, int64_t nbz) {
  __shared__ unsigned long long rx[16], rz[16];
  if (*(volatile int32_t*)&st->done) return;
  const int t = threadIdx.x;
  unsigned long long sx = 0, sz = 0;
  for (int64_t i = t; i < nbx; i += blockDim.x) sx += xpart[i];
  for (int64_t i = t; i < nbz; i += blockDim.x) sz += zpart[i];
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
    viol[k] = vx;
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

// Reduce the verification partials: max |y - x|, max(|Re|,|Im|) and the count above Delta.
__global__ void __launch_bounds__(1024) stats_kernel(DevState* st, const unsigned long long* vz, int64_t nbz,
                                                     const unsigned long long* vxc, const unsigned long long* vxm,
                                                     int64_t nbx) {
  __shared__ unsigned long long ra[16], rb[16], rc[16];
  const int t = threadIdx.x;
  unsigned long long a = 0, b = 0, c = 0;  // max bits of non-negative doubles order as integers
  for (int64_t i = t; i < nbz; i += blockDim.x) a = a > vz[i] ? a : vz[i];
  for (int64_t i = t; i < nbx; i += blockDim.x) {
    c += vxc[i];
    b = b > vxm[i] ? b : vxm[i];
  }
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
    unsigned long long A = 0, B = 0, Cc = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
      A = A > ra[w] ? A : ra[w];
      B = B > rb[w] ? B : rb[w];
      Cc += rc[w];
    }
    st->max_spatial_bits = A;
    st->max_spectral_bits = B;
    st->spectral_viol = Cc;
  }
}

// ---------------------------------------------------------------------------

struct Ctx {
  const Plan* p;
  char* ws;
  hipStream_t s;
  DevState* st() const { return (DevState*)(ws + p->off_state); }
  void* twT() const { return ws + p->off_twT; }
  void* tw64() const { return ws + p->off_tw64; }
  void* Z() const { return ws + p->off_Z; }
  void* A() const { return ws + p->off_A; }
  unsigned long long* part(int i) const { return (unsigned long long*)(ws + p->off_part) + (size_t)i * p->pmax; }
  // region indices
  static constexpr int PX = 0, PZ = 1, PVZ = 2, PVX = 3;  // PVX spans two regions (count, max)
};

hipError_t launch_ctl(const Ctx& c, unsigned long long* viol) {
  hipLaunchKernelGGL(ctl_kernel, dim3(1), dim3(1024), 0, c.s, c.st(), viol, c.part(Ctx::PX), c.p->nbx,
                     c.part(Ctx::PZ), c.p->nbz);
  return hipGetLastError();
}

hipError_t write_twiddles(const Ctx& c) {
  const Plan& p = *c.p;
  // table 0: working precision (read by the loop kernels); table 1: FP64 (verification)
  for (int tab = 0; tab < 2; ++tab) {
    const int dbl = (tab == 1 || p.dt == FFCZ_F64) ? 1 : 0;
    TwJobs jobs;
    memset(&jobs, 0, sizeof(jobs));
    jobs.dbl = dbl;
    int n = 0;
    jobs.j[n++] = TwJob{p.twz, p.H, p.Ez, 1};
    if (p.Ly) jobs.j[n++] = TwJob{p.twy, p.Ly, p.Ey, 0};
    jobs.j[n++] = TwJob{p.twx, p.Lx, p.Ex, 0};
    jobs.n = n;
    const int64_t tot = p.twT;
    const int nb = (int)((tot + 255) / 256);
    hipLaunchKernelGGL(twiddle_kernel, dim3(nb), dim3(256), 0, c.s, tab ? c.tw64() : c.twT(), jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Geometry of a strided-axis pass.
struct ColGeom {
  int L;
  int64_t outer, so, s;
  int64_t mrow_i, mrow_o;
};

ColGeom geom_y(const Plan& p, int64_t pitch) {
  return ColGeom{p.Ly, p.n[0], p.n[1] * pitch, pitch, 0, 0};
}
ColGeom geom_x(const Plan& p, int64_t pitch) {
  if (p.nd == 3) return ColGeom{p.Lx, p.n[1], pitch, p.n[1] * pitch, p.n[1], 1};
  return ColGeom{p.Lx, 1, 0, pitch, 1, 0};
}

template <typename T>
hipError_t run_col(int dt, int mode, const ColGeom& g, const Plan& p, const void* src, void* dst,
                   const void* tw, DevState* st, unsigned long long* part, uint8_t* fmask,
                   hipStream_t s) {
  ColArgs<T> a;
  memset(&a, 0, sizeof(a));
  const int C = col_block_cols(dt, g.L);
  a.src = (const cx<T>*)src;
  a.dst = (cx<T>*)dst;
  a.so = g.so;
  a.s = g.s;
  a.ncols = (int32_t)p.ncols;
  a.ncb = (int32_t)((p.ncols + C - 1) / C);
  a.tw = (const cx<T>*)tw;
  a.st = st;
  a.part = part;
  a.part_stride = p.pmax;
  a.fmask = fmask;
  a.f_plane = p.f_plane_bytes;
  a.f_row_bytes = p.f_row_bytes;
  a.mrow_i = g.mrow_i;
  a.mrow_o = g.mrow_o;
  const int64_t nb = g.outer * a.ncb;
  return launch_col(dt, mode, g.L, &a, nb, s);
}

template <typename T, typename TIO>
hipError_t run_row(int tdt, int iodt, int mode, const Plan& p, int64_t pitch, const void* src, void* dst,
                   const void* x, const void* xb, void* y, const void* tw, DevState* st,
                   unsigned long long* part, uint32_t* smask, hipStream_t s) {
  RowArgs<T, TIO> a;
  memset(&a, 0, sizeof(a));
  a.src = (const cx<T>*)src;
  a.dst = (cx<T>*)dst;
  a.pitch = pitch;
  a.nrows = p.nrows;
  a.x = (const TIO*)x;
  a.xb = (const TIO*)xb;
  a.y = (TIO*)y;
  a.tw = (const cx<T>*)tw;
  a.st = st;
  a.part = part;
  a.smask = smask;
  a.s_plane = p.s_plane_bytes / 4;
  a.s_row_w32 = (int32_t)p.s_row_w32;
  const int R = row_block_rows(p.H);
  const int64_t nb = (p.nrows + R - 1) / R;
  if (mode == ROW_VERIFY && tdt == 1 && iodt == 0) return launch_row_verify_f32io(p.H, &a, nb, s);
  return tdt == 0 ? launch_row_f32(mode, p.H, &a, nb, s) : launch_row_f64(mode, p.H, &a, nb, s);
}

template <typename T>
hipError_t row_T(int mode, const Ctx& c, const void* src, void* dst, const void* x, const void* xb, void* y,
                 uint32_t* smask) {
  const Plan& p = *c.p;
  const void* tw = (const char*)c.twT() + sizeof(cx<T>) * p.twz;
  return run_row<T, T>(p.dt, p.dt, mode, p, p.pitch, src, dst, x, xb, y, tw, c.st(), c.part(Ctx::PZ), smask, c.s);
}

template <typename T>
hipError_t enqueue_round(const Ctx& c, int r, unsigned long long* viol, uint8_t* fmask, uint32_t* smask) {
  unsigned long long* px = c.part(Ctx::PX);
  const Plan& p = *c.p;
  const char* twb = (const char*)c.twT();
  const void* twy = twb + sizeof(cx<T>) * p.twy;
  const void* twx = twb + sizeof(cx<T>) * p.twx;
  hipError_t e;
  if (p.nd == 3) {
    e = timed(PK_YFWD, r, c.s, [&] {
      return run_col<T>(p.dt, COL_FWD, geom_y(p, p.pitch), p, c.Z(), c.A(), twy, c.st(), px, fmask, c.s);
    });
    if (e != hipSuccess) return e;
    e = timed(PK_XPASS, r, c.s, [&] {
      return run_col<T>(p.dt, COL_XPASS, geom_x(p, p.pitch), p, c.A(), c.A(), twx, c.st(), px, fmask, c.s);
    });
    if (e != hipSuccess) return e;
    e = launch_ctl(c, viol);
    if (e != hipSuccess) return e;
    e = timed(PK_YINV, r, c.s, [&] {
      return run_col<T>(p.dt, COL_INV, geom_y(p, p.pitch), p, c.A(), c.A(), twy, c.st(), px, fmask, c.s);
    });
    if (e != hipSuccess) return e;
  } else {
    e = timed(PK_XPASS, r, c.s, [&] {
      return run_col<T>(p.dt, COL_XPASS, geom_x(p, p.pitch), p, c.Z(), c.A(), twx, c.st(), px, fmask, c.s);
    });
    if (e != hipSuccess) return e;
    e = launch_ctl(c, viol);
    if (e != hipSuccess) return e;
  }
  return timed(PK_ZPASS, r, c.s, [&] { return row_T<T>(ROW_LOOP, c, c.A(), c.Z(), nullptr, nullptr, nullptr, smask); });
}

template <typename T>
hipError_t enqueue_verify(const Ctx& c, const void* x, const void* y) {
  const Plan& p = *c.p;
  const char* tb = (const char*)c.tw64();
  void* W = c.Z();  // FP64 spectrum over Z..A
  hipError_t e = timed(PK_VZ, -1, c.s, [&] {
    return run_row<double, T>(1, p.dt, ROW_VERIFY, p, p.pitch64, nullptr, W, x, y, nullptr, tb + 16 * p.tw64z,
                              c.st(), c.part(Ctx::PVZ), nullptr, c.s);
  });
  if (e != hipSuccess) return e;
  if (p.nd == 3) {
    e = timed(PK_VY, -1, c.s, [&] {
      return run_col<double>(1, COL_FWD_NS, geom_y(p, p.pitch64), p, W, W, tb + 16 * p.tw64y, c.st(),
                             c.part(Ctx::PVX), nullptr, c.s);
    });
    if (e != hipSuccess) return e;
  }
  e = timed(PK_VX, -1, c.s, [&] {
    return run_col<double>(1, COL_VERIFY, geom_x(p, p.pitch64), p, W, W, tb + 16 * p.tw64x, c.st(),
                           c.part(Ctx::PVX), nullptr, c.s);
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(1024), 0, c.s, c.st(), c.part(Ctx::PVZ), p.nbz, c.part(Ctx::PVX),
                     c.part(Ctx::PVX + 1), p.nbvx);
  return hipGetLastError();
}

// pinned host mirror of the device state (one per thread)
struct HostMirror {
  DevState* st = nullptr;
  unsigned long long* v = nullptr;
  ~HostMirror() {
    if (st) (void)hipHostFree(st);
    if (v) (void)hipHostFree(v);
  }
};
thread_local HostMirror g_mirror;

hipError_t mirror() {
  if (!g_mirror.st) {
    hipError_t e = hipHostMalloc((void**)&g_mirror.st, sizeof(DevState), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipHostMalloc((void**)&g_mirror.v, 2 * sizeof(unsigned long long), hipHostMallocDefault);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

double default_mu(int dt) { return dt == FFCZ_F64 ? std::ldexp(1.0, -16) : 0.0; }

template <typename T>
int32_t correct_impl(const Plan& p, const void* x, const void* xb, void* y, double E, double D, int32_t max_iter,
                     const ffcz_options& o, void* ws, hipStream_t s, ffcz_stats* stats) {
  Ctx c{&p, (char*)ws, s};
  unsigned long long* viol = o.viol_per_round ? (unsigned long long*)o.viol_per_round
                                              : (unsigned long long*)((char*)ws + p.off_viol);
  double mu = o.margin_rel;
  if (!(mu > 0.0)) {
    if (p.dt == FFCZ_F64) {
      mu = default_mu(p.dt);
    } else {
      int32_t st = ffcz_suggest_margin(p.dt, p.nd, p.n, x, D, ws, p.bytes, s, &mu);
      if (st != FFCZ_OK) return st;
    }
  }
  if (!(mu < 1.0)) return fail(FFCZ_E_INVALID, "margin_rel must be in [0, 1)");
  const bool rec = o.masks_out != nullptr;
  uint32_t* smask = rec ? (uint32_t*)o.masks_out : nullptr;
  uint8_t* fmask = rec ? (uint8_t*)o.masks_out + (size_t)(max_iter + 1) * p.s_plane_bytes : nullptr;

  StateInit si;
  si.E = E;
  si.Ep = E * (1.0 - mu);
  si.Delta = D;
  si.Dp = D * (1.0 - mu);
  si.inv_n = 1.0 / (double)p.N;
  si.max_iter = max_iter;
  si.fixed = o.fixed_iterations ? 1 : 0;
  si.record_masks = rec ? 1 : 0;
  hipLaunchKernelGGL(state_init_kernel, dim3(std::max(1, (max_iter + 2 + 255) / 256)), dim3(256), 0, s, c.st(),
                     viol, max_iter + 1, si);
  HIPCHK(hipGetLastError());
  HIPCHK(write_twiddles(c));
  HIPCHK(timed(PK_INIT, -1, s, [&] { return row_T<T>(ROW_INIT, c, nullptr, c.Z(), x, xb, nullptr, smask); }));

  const int chunk = o.graph_chunk > 0 ? o.graph_chunk : 4;
  HIPCHK(mirror());
  int enq = 0;
  const bool sync_needed = !(o.fixed_iterations && stats == nullptr);
  if (o.fixed_iterations) {
    // exactly max_iter blocks plus the final check: no polling needed
    for (int r = 0; r <= max_iter; ++r) HIPCHK(enqueue_round<T>(c, r, viol, fmask, smask));
  } else {
    for (;;) {
      for (int r = 0; r < chunk; ++r) HIPCHK(enqueue_round<T>(c, enq + r, viol, fmask, smask));
      enq += chunk;
      HIPCHK(hipMemcpyAsync(g_mirror.st, c.st(), sizeof(DevState), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (g_mirror.st->done) break;
      if (enq > max_iter + 2 * chunk + 2)
        return fail(FFCZ_E_HIP, "loop did not report completion (device state inconsistent)");
    }
  }
  HIPCHK(timed(PK_FINAL, -1, s, [&] { return row_T<T>(ROW_FINAL, c, c.Z(), nullptr, x, nullptr, y, nullptr); }));
  if (o.verify_fp64) HIPCHK(enqueue_verify<T>(c, x, y));
  if (!sync_needed) {
    prof_settle(max_iter);
    return FFCZ_OK;
  }
  HIPCHK(hipMemcpyAsync(g_mirror.st, c.st(), sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const DevState h = *g_mirror.st;
  prof_settle(h.round);
  HIPCHK(hipMemcpyAsync(&g_mirror.v[0], viol, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&g_mirror.v[1], viol + h.round, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->rounds = h.round;
    stats->converged = h.converged;
    stats->f_viol_initial = (int64_t)g_mirror.v[0];
    stats->f_viol_final = (int64_t)g_mirror.v[1];
    stats->s_clipped_total = (int64_t)h.s_clipped_total;
    stats->s_guard = (int64_t)h.s_guard;
    stats->nonfinite = (int64_t)h.nonfinite;
    double ms, mf;
    unsigned long long b1 = h.max_spatial_bits, b2 = h.max_spectral_bits;
    memcpy(&ms, &b1, 8);
    memcpy(&mf, &b2, 8);
    stats->max_spatial_err = o.verify_fp64 ? ms : NAN;
    stats->max_spectral_err = o.verify_fp64 ? mf : NAN;
    stats->spectral_viol = (int64_t)h.spectral_viol;
    stats->margin_used = mu;
  }
  if (h.nonfinite) return fail(FFCZ_E_NONFINITE, "x or x_hat holds NaN or Inf");
  if (!h.converged && !o.fixed_iterations) return FFCZ_NOT_CONVERGED;
  if (o.verify_fp64) {
    double ms, mf;
    unsigned long long b1 = h.max_spatial_bits, b2 = h.max_spectral_bits;
    memcpy(&ms, &b1, 8);
    memcpy(&mf, &b2, 8);
    if (!(ms <= E) || !(mf <= D)) {
      g_err = "FP64 re-verification failed";
      return FFCZ_VERIFY_FAILED;
    }
  }
  return FFCZ_OK;
}

template <typename T>
int32_t backward_impl(const Plan& p, int32_t rounds, const void* masks, const void* gy, void* gb, void* ws,
                      hipStream_t s) {
  Ctx c{&p, (char*)ws, s};
  StateInit si;
  memset(&si, 0, sizeof(si));
  si.inv_n = 1.0 / (double)p.N;
  si.max_iter = rounds;
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, c.st(), (unsigned long long*)((char*)ws + p.off_viol),
                     1, si);
  HIPCHK(hipGetLastError());
  HIPCHK(write_twiddles(c));
  const char* mb = (const char*)masks;
  auto splane = [&](int k) { return (uint32_t*)(mb + (size_t)k * p.s_plane_bytes); };
  auto fplane = [&](int k) { return (uint8_t*)(mb + (size_t)(rounds + 1) * p.s_plane_bytes + (size_t)(k - 1) * 2 * p.f_plane_bytes); };
  const char* twb = (const char*)c.twT();
  const void* twy = twb + sizeof(cx<T>) * p.twy;
  const void* twx = twb + sizeof(cx<T>) * p.twx;
  if (rounds == 0) {
    // y = x + M_s^0 (x_hat - x): the gradient is the guard mask times dL/dy
    HIPCHK(row_T<T>(ROW_BINIT, c, nullptr, c.Z(), nullptr, gy, nullptr, splane(0)));
    HIPCHK(row_T<T>(ROW_BFINAL, c, c.Z(), nullptr, nullptr, nullptr, gb, splane(0)));
    // ROW_BFINAL applies the mask a second time; masks are idempotent
    return FFCZ_OK;
  }
  HIPCHK(timed(PK_BZ, -1, s, [&] { return row_T<T>(ROW_BINIT, c, nullptr, c.Z(), nullptr, gy, nullptr, splane(rounds)); }));
  for (int k = rounds; k >= 1; --k) {
    if (p.nd == 3)
      HIPCHK(timed(PK_BY, -1, s, [&] {
        return run_col<T>(p.dt, COL_FWD_NS, geom_y(p, p.pitch), p, c.Z(), c.Z(), twy, c.st(), nullptr, nullptr, s);
      }));
    HIPCHK(timed(PK_BX, -1, s, [&] {
      return run_col<T>(p.dt, COL_XBACK, geom_x(p, p.pitch), p, c.Z(), c.Z(), twx, c.st(), nullptr, fplane(k), s);
    }));
    if (p.nd == 3)
      HIPCHK(timed(PK_BY, -1, s, [&] {
        return run_col<T>(p.dt, COL_INV_NS, geom_y(p, p.pitch), p, c.Z(), c.Z(), twy, c.st(), nullptr, nullptr, s);
      }));
    if (k > 1)
      HIPCHK(timed(PK_BZ, -1, s, [&] { return row_T<T>(ROW_BLOOP, c, c.Z(), c.Z(), nullptr, nullptr, nullptr, splane(k - 1)); }));
    else
      HIPCHK(timed(PK_BZ, -1, s, [&] { return row_T<T>(ROW_BFINAL, c, c.Z(), nullptr, nullptr, nullptr, gb, splane(0)); }));
  }
  return FFCZ_OK;
}

}  // namespace

extern "C" {

int32_t ffcz_version(void) { return 100; }

void ffcz_profile_enable(int32_t on) {
  g_prof.on = on != 0;
  for (int k = 0; k < PK_COUNT; ++k) {
    g_prof.ms[k] = 0.0;
    g_prof.cnt[k] = 0;
  }
}

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

const char* ffcz_last_error(void) { return g_err.c_str(); }

void ffcz_default_options(ffcz_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->verify_fp64 = 1;
  o->graph_chunk = 4;
}

size_t ffcz_workspace_bytes(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t max_iter) {
  Plan p;
  std::string keep = g_err;
  if (make_plan(dtype, ndim, shape, max_iter < 0 ? 0 : max_iter, p) != FFCZ_OK) return 0;
  g_err = keep;
  return p.bytes;
}

size_t ffcz_mask_bytes(int32_t ndim, const int64_t* shape, int32_t rounds) {
  Plan p;
  std::string keep = g_err;
  if (rounds < 0 || make_plan(FFCZ_F32, ndim, shape, rounds, p) != FFCZ_OK) return 0;
  g_err = keep;
  return (size_t)(rounds + 1) * p.s_plane_bytes + (size_t)rounds * 2 * p.f_plane_bytes;
}

int32_t ffcz_suggest_margin(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, double delta_f,
                            void* ws, size_t ws_bytes, void* stream, double* mu_out) {
  Plan p;
  int32_t r = make_plan(dtype, ndim, shape, 0, p);
  if (r != FFCZ_OK) return r;
  if (!x || !mu_out) return fail(FFCZ_E_INVALID, "null pointer");
  if (!std::isfinite(delta_f) || delta_f < 0) return fail(FFCZ_E_INVALID, "delta_f must be finite and >= 0");
  if (dtype == FFCZ_F64) {
    *mu_out = std::ldexp(1.0, -16);
    return FFCZ_OK;
  }
  if (!ws || ws_bytes < p.off_state + sizeof(DevState)) return fail(FFCZ_E_WORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  DevState* st = (DevState*)((char*)ws + p.off_state);
  StateInit si;
  memset(&si, 0, sizeof(si));
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, st, (unsigned long long*)nullptr, 0, si);
  HIPCHK(hipGetLastError());
  const int nb = (int)std::min<int64_t>(4096, (p.N + 255) / 256);
  hipLaunchKernelGGL(ulp_kernel<float>, dim3(nb), dim3(256), 0, s, (const float*)x, p.N, st);
  HIPCHK(hipGetLastError());
  HIPCHK(mirror());
  HIPCHK(hipMemcpyAsync(g_mirror.st, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double sigma = std::sqrt(g_mirror.st->ulp2_sum / (double)p.N / 12.0);
  double mu = delta_f > 0 ? 8.0 * sigma * std::sqrt((double)p.N / 2.0) / delta_f : 0.5;
  mu = std::min(0.5, std::max(std::ldexp(1.0, -16), mu));
  *mu_out = mu;
  return FFCZ_OK;
}

int32_t ffcz_correct(int32_t dtype, int32_t ndim, const int64_t* shape, const void* x, const void* xb, void* y,
                     double eps_s, double delta_f, int32_t max_iter, const ffcz_options* opts, void* ws,
                     size_t ws_bytes, void* stream, ffcz_stats* stats) {
  Plan p;
  int32_t r = make_plan(dtype, ndim, shape, max_iter, p);
  if (r != FFCZ_OK) return r;
  if (!x || !xb || !y) return fail(FFCZ_E_INVALID, "null data pointer");
  if (x == xb || x == y) return fail(FFCZ_E_INVALID, "x_orig must not alias x_base or x_out");
  if (!std::isfinite(eps_s) || eps_s < 0) return fail(FFCZ_E_INVALID, "eps_s must be finite and >= 0");
  if (!std::isfinite(delta_f) || delta_f < 0) return fail(FFCZ_E_INVALID, "delta_f must be finite and >= 0");
  if (!ws || ws_bytes < p.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_workspace_bytes()");
  if (((uintptr_t)ws & 255) || ((uintptr_t)x & 15) || ((uintptr_t)xb & 15) || ((uintptr_t)y & 15))
    return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte and data 16-byte aligned");
  ffcz_options o;
  if (opts) o = *opts;
  else ffcz_default_options(&o);
  if (o.fixed_iterations && o.masks_out && p.dt == FFCZ_F64 && col_block_cols(1, p.Lx) < 8)
    return fail(FFCZ_E_SHAPE, "mask recording needs at least 8 columns per block");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == FFCZ_F32) return correct_impl<float>(p, x, xb, y, eps_s, delta_f, max_iter, o, ws, s, stats);
  return correct_impl<double>(p, x, xb, y, eps_s, delta_f, max_iter, o, ws, s, stats);
}

int32_t ffcz_correct_backward(int32_t dtype, int32_t ndim, const int64_t* shape, int32_t rounds, const void* masks,
                              const void* gy, void* gb, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int32_t r = make_plan(dtype, ndim, shape, rounds, p);
  if (r != FFCZ_OK) return r;
  if (!masks || !gy || !gb) return fail(FFCZ_E_INVALID, "null pointer");
  if (!ws || ws_bytes < p.bytes) return fail(FFCZ_E_WORKSPACE, "workspace smaller than ffcz_workspace_bytes()");
  if ((uintptr_t)ws & 255) return fail(FFCZ_E_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == FFCZ_F32) return backward_impl<float>(p, rounds, masks, gy, gb, ws, s);
  return backward_impl<double>(p, rounds, masks, gy, gb, ws, s);
}

}  // extern "C"
