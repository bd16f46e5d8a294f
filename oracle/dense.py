"""Brute-force O(N^2) version of the correction loop (test infrastructure only).

The DFT is written out as an explicit matrix from Eq. 1 (1D) and its
multidimensional form (Sec. III, 2D DFT), with the phase reduced exactly in
integers: ``W[k, n] = exp(-2 pi i ((k n) mod L) / L)``.  Eq. 2 is stated over
the FULL spectrum, so this version checks and clips all ``N`` coefficients and
inverts with the conjugate-transposed matrix.  It pins the half-spectrum FFT
loop of ``oracle.ffcz`` on grids with ``N <= ~600``.
"""

from __future__ import annotations

import numpy as np

from .ffcz import DEFAULT_MU


def dft_matrix_1d(n: int) -> np.ndarray:
    k = np.arange(n, dtype=np.int64)
    ph = np.outer(k, k) % n
    return np.exp(-2j * np.pi * ph / n)


def dft_matrix(shape) -> np.ndarray:
    """Full N x N DFT matrix for a C-ordered field (last axis fastest)."""
    W = np.ones((1, 1), dtype=np.complex128)
    for n in shape:
        W = np.kron(W, dft_matrix_1d(n))
    return W


def half_spectrum_indices(shape) -> np.ndarray:
    """Flat indices (into the full C-ordered spectrum) of the entries a real
    transform keeps: last-axis frequency ``0 .. n_last//2``."""
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    return idx[..., : shape[-1] // 2 + 1].ravel()


def clip_box(v: np.ndarray, b: float) -> np.ndarray:
    """Euclidean projection onto the box ``[-b, b]`` per coordinate (Eq. 2, third line):
    every coordinate beyond the bound is set to the bound, the rest are kept."""
    out = np.array(v, dtype=np.float64, copy=True)
    out[out > b] = b
    out[out < -b] = -b
    return out


def dense_fft(eps: np.ndarray) -> np.ndarray:
    """Full spectrum of a real field via the explicit DFT matrix (Eq. 3)."""
    W = dft_matrix(eps.shape)
    return (W @ eps.ravel().astype(np.complex128)).reshape(eps.shape)


def dense_correct(x, xb, E: float, Delta: float, max_iter: int, mu: float = DEFAULT_MU):
    """Alg. 1 with dense matrices.  Returns ``(eps, rounds, viol_half, viol_full, max_imag)``.

    ``viol_half`` counts violating coefficients of the half-spectrum (the count
    the FFT oracle reports); ``viol_full`` counts them over all N coefficients.
    ``max_imag`` is the largest imaginary part met after an inverse transform
    (zero up to rounding when the full-spectrum clip stays Hermitian).
    """
    shape = x.shape
    N = int(np.prod(shape))
    W = dft_matrix(shape)
    Winv = W.conj().T / N
    half = half_spectrum_indices(shape)
    Ep = E * (1.0 - mu)
    Dp = Delta * (1.0 - mu)
    eps = (np.asarray(xb, np.float64) - np.asarray(x, np.float64)).ravel()
    eps = clip_box(eps, Ep)
    vh, vf = [], []
    max_imag = 0.0
    k = 0
    while True:
        d = W @ eps
        bad = (np.abs(d.real) > Delta) | (np.abs(d.imag) > Delta)
        vh.append(int(np.count_nonzero(bad[half])))
        vf.append(int(np.count_nonzero(bad)))
        if vf[-1] == 0 or k == max_iter:
            break
        d = clip_box(d.real, Dp) + 1j * clip_box(d.imag, Dp)
        e = Winv @ d
        max_imag = max(max_imag, float(np.max(np.abs(e.imag))))
        eps = clip_box(e.real, Ep)
        k += 1
    return eps.reshape(shape), k, vh, vf, max_imag


def dense_correct_edits(x, xb, Ep: float, Dc: float, Dp: float, max_iter: int):
    """Alg. 1 with dense matrices and its edit bookkeeping over the FULL spectrum.

    The check counts ``|Re|, |Im| > Dc``, the f-projection clips to ``Dp`` and the
    s-projection to ``Ep`` (the guard clip first).  Returns ``(eps, rounds,
    spat_edits, freq_edits)``: every s-clip displacement summed per point (guard
    included) and every f-clip displacement summed per coefficient, all N of them.
    """
    shape = x.shape
    N = int(np.prod(shape))
    W = dft_matrix(shape)
    Winv = W.conj().T / N
    raw = (np.asarray(xb, np.float64) - np.asarray(x, np.float64)).ravel()
    eps = clip_box(raw, Ep)
    spat = eps - raw
    freq = np.zeros(N, dtype=np.complex128)
    k = 0
    while True:
        d = W @ eps
        bad = (np.abs(d.real) > Dc) | (np.abs(d.imag) > Dc)
        if not np.any(bad) or k == max_iter:
            break
        dc = clip_box(d.real, Dp) + 1j * clip_box(d.imag, Dp)
        freq += dc - d
        e = (Winv @ dc).real
        eps = clip_box(e, Ep)
        spat += eps - e
        k += 1
    return eps.reshape(shape), k, spat.reshape(shape), freq.reshape(shape)
