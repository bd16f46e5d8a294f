"""Seeded synthetic inputs shaped like the paper's datasets.

This module only draws inputs: it holds none of the correction's arithmetic
and is shared by the tests and the benchmark.  The fields stand in for the
datasets of Table 1 (Nyx cosmology density, S3D combustion, HEDM diffraction,
EEG), which are not available; nothing from those datasets is reproduced.

Recipes
-------
``grf``       Gaussian random field with isotropic power spectrum ``|k|^-alpha``:
              white N(0,1) noise, real FFT, amplitude ``|k|^(-alpha/2)`` on the
              signed integer frequencies (0 at k = 0), inverse FFT, then
              standardised to mean 0 and standard deviation 1.
``lognormal`` ``exp(grf)`` (a density-like, positive, skewed field).
``quantize``  the base-compressor stand-in: uniform scalar quantiser with bin
              ``2E`` (``2E * rint(x / 2E)``, half to even), which honours ``|x_hat - x| <= E``.
``spatial_bound``  ``E = r * (max x - min x)`` over the dtype-cast field.
``spectral_bound`` ``Delta`` = q-th percentile (linear interpolation) of
              ``max(|Re D_k|, |Im D_k|)`` over the half-spectrum of ``D = DFT(x_hat - x)``
              (moved halfway to the next distinct value if it equals a coefficient),
              so that about ``(100 - q)%`` of the coefficients start out violating.
"""

from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np
import scipy.fft as sfft


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _kmag(shape) -> np.ndarray:
    axes = []
    for i, n in enumerate(shape):
        if i == len(shape) - 1:
            f = np.arange(n // 2 + 1, dtype=np.float64)
        else:
            f = np.fft.fftfreq(n) * n
        sh = [1] * len(shape)
        sh[i] = f.size
        axes.append((f * f).reshape(sh))
    k2 = axes[0]
    for a in axes[1:]:
        k2 = k2 + a
    return np.sqrt(k2)


def grf(shape, alpha: float, seed: int) -> np.ndarray:
    """FP64 Gaussian random field with P(k) proportional to |k|^-alpha."""
    shape = tuple(int(n) for n in shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    W = sfft.rfftn(w, workers=_workers())
    del w
    k = _kmag(shape)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** (-alpha / 2.0), 0.0)
    W *= amp
    del amp, k
    f = sfft.irfftn(W, s=shape, workers=_workers())
    del W
    f -= f.mean()
    s = f.std()
    if s > 0:
        f /= s
    return f


def lognormal(shape, alpha: float, seed: int) -> np.ndarray:
    return np.exp(grf(shape, alpha, seed))


def quantize(x: np.ndarray, E: float) -> np.ndarray:
    """Uniform quantiser with bin 2E in FP64 (half to even)."""
    x64 = np.asarray(x, dtype=np.float64)
    if E <= 0:
        return x64.copy()
    return (2.0 * E) * np.rint(x64 / (2.0 * E))


def spatial_bound(x: np.ndarray, r: float) -> float:
    x64 = np.asarray(x, dtype=np.float64)
    return float(r * (x64.max() - x64.min()))


def spectral_bound(x: np.ndarray, xb: np.ndarray, q: float) -> float:
    d = np.asarray(xb, dtype=np.float64) - np.asarray(x, dtype=np.float64)
    D = sfft.rfftn(d, workers=_workers())
    m = np.maximum(np.abs(D.real), np.abs(D.imag)).ravel()
    p = float(np.percentile(m, q))
    # Conjugate pairs in the self-conjugate planes give equal values, so the
    # interpolated percentile can coincide with a coefficient; a bound sitting
    # exactly on a coefficient makes the violation count depend on rounding.
    # Move it halfway to the next larger distinct value instead.
    if np.any(m == p):
        above = m[m > p]
        if above.size:
            p = 0.5 * (p + float(above.min()))
    return p


@dataclasses.dataclass
class Problem:
    """One correction instance: original, base reconstruction, bounds, cap."""
    name: str
    x: np.ndarray
    xb: np.ndarray
    E: float
    Delta: float
    max_iter: int
    fixed: bool = False


def make_problem(name: str, x64: np.ndarray, dtype, r: float, q: float, max_iter: int,
                 fixed: bool = False) -> Problem:
    """Cast the field, quantise it with bin 2E and set E and Delta by the recipes above."""
    x = np.asarray(x64).astype(dtype)
    E = spatial_bound(x, r)
    xb = quantize(x, E).astype(dtype)
    Delta = spectral_bound(x, xb, q)
    return Problem(name, x, xb, E, Delta, max_iter, fixed)


# ---------------------------------------------------------------------------
# Configurations (seeds fixed).  ``n`` lets tests run the same recipe smaller.

def config_grf_fp64(n: int = 64) -> Problem:
    """64^3 FP64 GRF, P(k) ~ k^-2, E = 1e-3 x range, Delta at the 90th percentile, 200 rounds."""
    return make_problem(f"grf{n}_fp64", grf((n, n, n), 2.0, 1), np.float64, 1e-3, 90.0, 200)


def config_lognormal(n: int = 512, dtype=np.float32) -> Problem:
    """512^3 lognormal density (exp of a k^-2.5 GRF), E = 1e-4 x range, 95th percentile, 500 rounds."""
    tag = "fp32" if np.dtype(dtype) == np.float32 else "fp64"
    return make_problem(f"lognormal{n}_{tag}", lognormal((n, n, n), 2.5, 2), dtype, 1e-4, 95.0, 500)


def config_kolmogorov(n: int = 1024) -> Problem:
    """1024^3 FP32 turbulence-like component, |k|^-5/3 PSD, E = 1e-4 x range, 99th percentile."""
    return make_problem(f"kolmogorov{n}_fp32", grf((n, n, n), 5.0 / 3.0, 3), np.float32,
                        1e-4, 99.0, 500)


def config_grad(n: int = 256, rounds: int = 50) -> Problem:
    """256^3 FP32 GRF, k^-2, E = 1e-3 x range, 90th percentile, fixed 50 rounds."""
    return make_problem(f"grf{n}_fp32_grad", grf((n, n, n), 2.0, 5), np.float32, 1e-3, 90.0,
                        rounds, fixed=True)


def eeg_length(i: int, lo: int = 2 ** 12, hi: int = 2 ** 18) -> int:
    rng = np.random.default_rng(40000 + i)
    return int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def eeg_signal(i: int, length: Optional[int] = None, fs: float = 256.0) -> np.ndarray:
    """Pink (1/f) noise of unit std plus 1-3 alpha-band (8-13 Hz) sinusoids."""
    L = eeg_length(i) if length is None else int(length)
    rng = np.random.default_rng(40000 + i)
    rng.uniform()  # the draw used by eeg_length
    w = rng.standard_normal(L)
    W = np.fft.rfft(w)
    f = np.arange(W.size, dtype=np.float64)
    W *= np.where(f > 0, 1.0 / np.sqrt(np.maximum(f, 1.0)), 0.0)
    p = np.fft.irfft(W, n=L)
    s = p.std()
    if s > 0:
        p /= s
    t = np.arange(L) / fs
    for _ in range(int(rng.integers(1, 4))):
        fr = rng.uniform(8.0, 13.0)
        a = rng.uniform(0.5, 2.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        p += a * np.sin(2.0 * math.pi * fr * t + ph)
    return p


def diffraction_field(j: int, n: int = 2048) -> np.ndarray:
    """Poisson counts of an fftshifted far-field intensity of a random disk object."""
    rng = np.random.default_rng(50000 + j)
    rad = rng.uniform(n / 16.0, n / 4.0)
    yy, xx = np.mgrid[0:n, 0:n]
    disk = ((yy - n / 2) ** 2 + (xx - n / 2) ** 2) <= rad * rad
    amp = rng.uniform(0.0, 1.0, (n, n))
    ph = rng.uniform(0.0, 2.0 * math.pi, (n, n))
    obj = np.where(disk, amp * np.exp(1j * ph), 0.0)
    inten = np.abs(np.fft.fftshift(np.fft.fft2(obj))) ** 2
    inten *= 1e4 / inten.max()
    return rng.poisson(inten).astype(np.float64)


def config_eeg(i: int, length: Optional[int] = None) -> Problem:
    return make_problem(f"eeg{i}", eeg_signal(i, length), np.float32, 1e-3, 90.0, 200)


def config_diffraction(j: int, n: int = 2048) -> Problem:
    return make_problem(f"hedm{j}_{n}", diffraction_field(j, n), np.float32, 1e-3, 90.0, 200)
