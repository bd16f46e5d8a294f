// Set-up kernels of the generalised bounds (the footnote to Eq. 2 in Sec. IV-A; Sec. V-B,
// Observation 4): pointwise spectral bounds copied into the spectrum layout, their checks and
// minimum, and the pointwise bound that keeps every shell of the power spectrum within a
// relative error.
//
// Power-spectrum bound.  Shell b = rint(|k|) (|k| from the signed integer frequencies) holds
// P_b = sum w_k |X_k|^2 with full-spectrum weights w_k (2 for interior last-axis entries, 1 at
// k_z = 0 and at the Nyquist plane).  For an error with |Re|, |Im| <= D on every entry of the
// shell (box), |P_hat_b - P_b| <= 2 sqrt2 D S_b + 2 D^2 W_b with S_b = sum w_k |X_k| and
// W_b = sum w_k; for |delta_k| <= D (disk) it is at most 2 D S_b + D^2 W_b.  D_b is the
// positive root of that bound = rho P_b, computed as rho P_b / (sqrt(2 S^2 + 2 W rho P) +
// sqrt2 S) (box) or rho P_b / (sqrt(S^2 + W rho P) + S) (disk), which has no cancellation.
#pragma once
#include "common.hpp"

namespace ffcz {

constexpr int kMaxShells = 2560;  // rint(|k|) + 1 for every supported shape (at most 2,509)
constexpr int kMinSlots = 1024;   // block minima of a bound set

// Geometry of a half-spectrum laid out in rows of ncols entries, rows grouped in planes of
// 2^lg_rpp rows at a pitch / plane stride (complex entries).
struct SpecGeom {
  int64_t nrows;
  int32_t ncols, lg_rpp;
  int64_t pitch, plane;
  __device__ __forceinline__ int64_t addr(int64_t e) const {
    const int64_t r = e / ncols, col = e - r * ncols;
    return (r >> lg_rpp) * plane + (r & ((int64_t(1) << lg_rpp) - 1)) * pitch + col;
  }
};

// Bits of a non-negative double (they order as integers).
__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// The caller's spectral bounds (M entries in C order, or scalars when the arrays are null) as
// (Re, Im) pairs in the working type at the spectrum's layout.  A scalar is rounded toward zero
// in FP32 (the bound does not grow); arrays arrive in the working type.  bad counts entries
// that are negative or not finite; minpart[block] receives the block's smallest bound.
template <typename T>
__global__ void __launch_bounds__(256) bounds_setup_kernel(const T* dre, const T* dim, double sre, double sim,
                                                           cx<T>* out, int64_t M, SpecGeom g,
                                                           unsigned long long* minpart, unsigned long long* bad) {
  __shared__ unsigned long long red[4];
  unsigned long long mn = ~0ull, nbad = 0;
  const T cre = to_t<T>(sre), cim = to_t<T>(sim);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < M; e += (int64_t)gridDim.x * 256) {
    const T br = dre ? dre[e] : cre;
    const T bi = dim ? dim[e] : (dre && !dim ? br : cim);
    const bool ok = isfinite((double)br) && isfinite((double)bi) && br >= T(0) && bi >= T(0);
    nbad += ok ? 0 : 1;
    const double m = fmin((double)br, (double)bi);
    if (ok) mn = mn < dbits(m) ? mn : dbits(m);
    out[g.addr(e)] = cx<T>{br, bi};
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(mn, off, 64);
    mn = mn < o ? mn : o;
    nbad += __shfl_xor(nbad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  if ((threadIdx.x & 63) == 0 && nbad) atomicAdd(bad, nbad);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
    for (int w = 1; w < 4; ++w) m = m < red[w] ? m : red[w];
    minpart[blockIdx.x] = m;
  }
}

// Spatial bounds E_n: count entries that are negative or not finite.
template <typename T>
__global__ void __launch_bounds__(256) spatial_check_kernel(const T* E, int64_t n, unsigned long long* bad) {
  unsigned long long nbad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = (double)E[i];
    nbad += (isfinite(v) && v >= 0.0) ? 0 : 1;
  }
  for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off, 64);
  if ((threadIdx.x & 63) == 0 && nbad) atomicAdd(bad, nbad);
}

// Per-shell sums of the FP64 spectrum W of x: each block adds its entries into LDS shells
// (atomic adds, so the order of the additions is not fixed), then stores its partial sums
// part[block][3][nb] (P, S, W).  Entry e = row * ncols + k_z; row = i0 (2D) or i0 n1 + i1 (3D).
__global__ void __launch_bounds__(256) shell_part_kernel(const cx<double>* W, SpecGeom g, int nd, int64_t n0,
                                                         int64_t n1, int64_t nl, int nb, double* part) {
  __shared__ double sh[3 * kMaxShells];
  for (int i = threadIdx.x; i < 3 * nb; i += 256) sh[i] = 0.0;
  __syncthreads();
  const int64_t M = g.nrows * g.ncols;
  auto sfreq = [](int64_t k, int64_t n) -> double { return (double)(k < (n + 1) / 2 ? k : k - n); };
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < M; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / g.ncols, kz = e - r * g.ncols;
    double k2 = (double)kz * (double)kz;
    if (nd == 3) {
      const double f0 = sfreq(r / n1, n0), f1 = sfreq(r % n1, n1);
      k2 += f0 * f0 + f1 * f1;
    } else if (nd == 2) {
      const double f0 = sfreq(r, n0);
      k2 += f0 * f0;
    }
    const int b = (int)rint(sqrt(k2));
    const double w = (kz == 0 || 2 * kz == nl) ? 1.0 : 2.0;
    const cx<double> X = W[g.addr(e)];
    const double a2 = X.re * X.re + X.im * X.im;
    atomicAdd(&sh[b], w * a2);
    atomicAdd(&sh[nb + b], w * sqrt(a2));
    atomicAdd(&sh[2 * nb + b], w);
  }
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * 3 * nb;
  for (int i = threadIdx.x; i < 3 * nb; i += 256) out[i] = sh[i];
}

// One lane per shell: add the block partials in block order and take D_b.
__global__ void __launch_bounds__(256) shell_bound_kernel(const double* part, int nblk, int nb, double rho,
                                                          int disk, double* bins) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  double P = 0.0, S = 0.0, Wt = 0.0;
  for (int k = 0; k < nblk; ++k) {
    const double* q = part + (int64_t)k * 3 * nb;
    P += q[b];
    S += q[nb + b];
    Wt += q[2 * nb + b];
  }
  const double den = disk ? sqrt(S * S + Wt * rho * P) + S : sqrt(2.0 * S * S + 2.0 * Wt * rho * P) + sqrt(2.0) * S;
  bins[b] = den > 0.0 ? rho * P / den : 0.0;
}

// The shell bound of every half-spectrum entry, in C order, in the field's dtype (rounded
// toward zero in FP32: the bound does not grow).
template <typename T>
__global__ void __launch_bounds__(256) shell_scatter_kernel(const double* bins, int64_t nrows, int32_t ncols, int nd,
                                                            int64_t n0, int64_t n1, T* out) {
  const int64_t M = nrows * ncols;
  auto sfreq = [](int64_t k, int64_t n) -> double { return (double)(k < (n + 1) / 2 ? k : k - n); };
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < M; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / ncols, kz = e - r * ncols;
    double k2 = (double)kz * (double)kz;
    if (nd == 3) {
      const double f0 = sfreq(r / n1, n0), f1 = sfreq(r % n1, n1);
      k2 += f0 * f0 + f1 * f1;
    } else if (nd == 2) {
      const double f0 = sfreq(r, n0);
      k2 += f0 * f0;
    }
    out[e] = to_t<T>(bins[(int)rint(sqrt(k2))]);
  }
}

}  // namespace ffcz
