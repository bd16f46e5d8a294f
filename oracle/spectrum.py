"""Shell-binned power spectrum and log-spectrum loss (test infrastructure only).

Sec. III ("Power spectrum") sums ``|X_k|^2`` over the frequencies at the same
distance from the origin.  Readings: ``|k|`` is taken from the signed integer
frequencies of every axis, a coefficient falls in bin ``b = rint(|k|)``, bins
``1..nbins`` are kept (the mean-removal step only touches the excluded DC
bin), and the half-spectrum is weighted by 2 for interior last-axis
frequencies so that the sum equals the full-spectrum sum.  The loss
``sum_b (log P_y(b) - log P_x(b))^2`` is the differentiation workload; its
gradient is derived in ``loss_grad``.
"""

from __future__ import annotations

import numpy as np

from .ffcz import fft, ifft


def shell_bins(shape):
    """Bin index ``rint(|k|)`` and Hermitian weight for every half-spectrum entry."""
    axes = []
    for i, n in enumerate(shape):
        if i == len(shape) - 1:
            f = np.arange(n // 2 + 1, dtype=np.float64)
        else:
            f = np.fft.fftfreq(n) * n
        axes.append(f)
    grids = np.meshgrid(*axes, indexing="ij")
    kk = np.sqrt(sum(g * g for g in grids))
    b = np.rint(kk).astype(np.int64)
    n_last = shape[-1]
    kz = np.arange(n_last // 2 + 1)
    w1 = np.where((kz == 0) | ((n_last % 2 == 0) & (kz == n_last // 2)), 1.0, 2.0)
    w = np.broadcast_to(w1, b.shape)
    return b, w


def power_spectrum(y: np.ndarray, nbins: int) -> np.ndarray:
    """``P(b) = sum_{rint|k| = b} |Y_k|^2`` over the full spectrum, b = 1..nbins."""
    Y = fft(np.asarray(y, np.float64))
    b, w = shell_bins(y.shape)
    p = np.bincount(b.ravel(), weights=(w * np.abs(Y) ** 2).ravel(), minlength=nbins + 1)
    return p[1:nbins + 1]


def loss(y: np.ndarray, x: np.ndarray, nbins: int) -> float:
    d = np.log(power_spectrum(y, nbins)) - np.log(power_spectrum(x, nbins))
    return float(np.sum(d * d))


def loss_grad(y: np.ndarray, x: np.ndarray, nbins: int) -> np.ndarray:
    """Gradient of ``loss`` with respect to ``y``.

    ``dP_b/dy_n = 2 Re sum_{k in b} conj(Y_k) e^{-2 pi i k.n/N}``.  With
    ``a_k = 2 (log P_y - log P_x)(b_k) / P_y(b_k)`` (zero outside bins 1..nbins),
    symmetric in ``k -> -k``, the sum is ``N * IDFT(a Y)``, so the gradient is
    ``2 N irfftn(a Y)``.
    """
    y = np.asarray(y, np.float64)
    Y = fft(y)
    b, _ = shell_bins(y.shape)
    py = power_spectrum(y, nbins)
    px = power_spectrum(x, nbins)
    coef = np.zeros(nbins + 1)
    coef[1:] = 2.0 * (np.log(py) - np.log(px)) / py
    bb = np.where(b <= nbins, b, 0)
    a = np.where(b <= nbins, coef[bb], 0.0)
    return 2.0 * y.size * ifft(a * Y, y.shape)
