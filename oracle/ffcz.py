"""FP64 CPU oracle of the FFCz alternating projection (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

What is computed (paper Sec. IV):

* the spatial error ``eps = x_hat - x`` (Alg. 1, first statement; Sec. IV-A);
* its frequency error ``delta = DFT(eps)``, unnormalised with the ``e^{-i...}``
  sign of Eq. 1, which equals ``X_hat - X`` by Eq. 3;
* the s-cube ``|eps_n| <= E`` and the f-cube ``|Re delta_k|, |Im delta_k| <= Delta``
  of Eq. 2 / Eq. 4;
* the loop of Alg. 1: FFT, CheckConvergence, ProjectOntoFCube (clip Re and Im),
  IFFT, ProjectOntoSCube (clip eps), until no frequency component violates.

Readings taken where the paper is silent:

* Projections use the bounds shrunk by ``(1 - mu)`` with ``mu = 2**-16`` (the
  ``m = 16`` shrink of Sec. IV-B), while the check uses the unshrunk bounds.
  Without the shrink the loop need not terminate.
* A guard clip puts the initial error inside the shrunk s-cube (Sec. IV-B
  assumes the base output already lies in the s-cube).
* Only the half-spectrum of a real transform is stored and clipped; Hermitian
  symmetry (Sec. IV-A, "Frequency and spatial bases") makes this equal to the
  clip of the full spectrum.
* ``rounds`` counts completed projection blocks; the check after the last block
  always runs; ``max_iter`` caps the blocks.
* A violation is ``|v| > Delta`` (strict); a component is clipped when
  ``|v| > bound*(1-mu)``; a mask bit is 1 iff the component was left unclipped.
* FP32 outputs: ``y = x + eps`` is formed in FP64, rounded to nearest FP32 and
  then moved one ulp at a time toward ``x`` while ``|y - x| > E`` (closing clamp).
* Adjoint: each round is ``eps -> P_s(F^-1 P_f F eps)``; with frozen clip masks
  its transpose is ``M_s^{k-1} (F^-1 M_f^k F)``, applied in reverse order.
"""

from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional

import numpy as np
import scipy.fft as sfft

# Status codes mirror the C ABI.
OK = 0
NOT_CONVERGED = 1
VERIFY_FAILED = 2
E_INVALID = -1
E_SHAPE = -2
E_NONFINITE = -4

DEFAULT_MU = 2.0 ** -16  # m = 16 quantisation shrink (Sec. IV-B)

_WORKERS = 1


def set_workers(n: int) -> None:
    """Number of threads scipy.fft may use for the oracle's transforms."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def workers() -> int:
    return _WORKERS


class OracleError(ValueError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def fft(eps: np.ndarray) -> np.ndarray:
    """Unnormalised forward DFT of a real field, half-spectrum along the last axis (Eq. 1)."""
    return sfft.rfftn(eps, workers=_WORKERS)


def ifft(delta: np.ndarray, shape) -> np.ndarray:
    """Inverse of ``fft`` (the 1/N factor included), real output of ``shape``."""
    return sfft.irfftn(delta, s=tuple(shape), workers=_WORKERS)


def count_violations(delta: np.ndarray, Delta: float) -> int:
    """CheckConvergence (Alg. 1): number of half-spectrum entries with
    ``|Re| > Delta`` or ``|Im| > Delta`` (Eq. 2, second line)."""
    bad = (np.abs(delta.real) > Delta) | (np.abs(delta.imag) > Delta)
    return int(np.count_nonzero(bad))


def project_f(delta: np.ndarray, Dp: float):
    """ProjectOntoFCube (Alg. 1; Sec. IV-E): clip Re and Im separately to
    ``[-Dp, Dp]``.  Returns the clipped spectrum and the two keep-masks."""
    re = delta.real
    im = delta.imag
    keep_re = np.abs(re) <= Dp
    keep_im = np.abs(im) <= Dp
    out = np.clip(re, -Dp, Dp) + 1j * np.clip(im, -Dp, Dp)
    return out, keep_re, keep_im


def project_s(eps: np.ndarray, Ep: float):
    """ProjectOntoSCube (Alg. 1): clip every spatial error to ``[-Ep, Ep]``.
    Returns the clipped error, the keep-mask and the number of clipped entries."""
    keep = np.abs(eps) <= Ep
    return np.clip(eps, -Ep, Ep), keep, int(eps.size - np.count_nonzero(keep))


def ulp32(x: np.ndarray) -> np.ndarray:
    """Spacing of the FP32 grid at |x| (the rounding step of an FP32 output)."""
    return np.spacing(np.abs(np.asarray(x, dtype=np.float32))).astype(np.float64)


def suggest_margin(x: np.ndarray, Delta: float) -> float:
    """Relative shrink ``mu`` for an FP32 output.

    Rounding ``y = x + eps`` to FP32 adds an error of variance ``ulp^2/12`` per
    point; by Eq. 3 each Re/Im spectral component then moves by a sum of N such
    terms with weights cos/sin, whose standard deviation is about
    ``sigma_r * sqrt(N/2)``.  The margin keeps 8 of those inside the shrunk
    f-cube, and never goes below the paper's ``2^-16``.
    """
    x = np.asarray(x)
    n = x.size
    u = ulp32(x)
    sigma = math.sqrt(float(np.mean(u * u)) / 12.0)
    if Delta <= 0.0:
        return 0.5
    mu = 8.0 * sigma * math.sqrt(n / 2.0) / Delta
    return float(min(0.5, max(DEFAULT_MU, mu)))


def spectral_thresholds(Delta: float, mu: float, out_dtype) -> tuple:
    """``(Delta_c, Delta_p)``: the bound the check compares with and the bound the
    f-projection clips to.

    FP64 output: the check uses Delta itself and the projection the shrunk
    ``Delta (1 - mu)`` (Sec. IV-B).  FP32 output: rounding ``y`` moves every
    component by up to the margin's 8 standard deviations (``mu Delta``), and a
    coefficient the check accepted in ``(Delta_p, Delta]`` is never clipped, so the
    check itself runs ``mu Delta`` below Delta and the projection another
    ``mu Delta`` below the check.
    """
    rho = 0.0 if np.dtype(out_dtype) == np.float64 else float(mu)
    return Delta * (1.0 - rho), Delta * (1.0 - rho - mu)


def closing_clamp(y32: np.ndarray, x: np.ndarray, E: float) -> np.ndarray:
    """Move each FP32 output one ulp at a time toward ``x`` until
    ``|(double)y - (double)x| <= E`` holds in FP64."""
    y32 = np.array(y32, dtype=np.float32, copy=True)
    x64 = np.asarray(x, dtype=np.float64)
    xs = np.asarray(x, dtype=np.float32)
    bad = np.abs(y32.astype(np.float64) - x64) > E
    while np.any(bad):
        idx = np.nonzero(bad)
        y32[idx] = np.nextafter(y32[idx], xs[idx])
        bad = np.abs(y32.astype(np.float64) - x64) > E
    return y32


def verify(x: np.ndarray, y: np.ndarray, E: float, Delta: float):
    """FP64 re-verification of both bounds of Eq. 2 on an output ``y``.

    Returns ``(max|y-x|, max(|Re|,|Im|) of DFT(y-x), spectral violations, ok)``.
    """
    d = np.asarray(y, dtype=np.float64) - np.asarray(x, dtype=np.float64)
    ms = float(np.max(np.abs(d))) if d.size else 0.0
    D = fft(d)
    mf = float(max(np.max(np.abs(D.real)), np.max(np.abs(D.imag)))) if D.size else 0.0
    nv = count_violations(D, Delta)
    return ms, mf, nv, (ms <= E and mf <= Delta)


@dataclasses.dataclass
class Masks:
    """Clip keep-masks recorded along the trajectory (1 = left unclipped).

    ``s[0]`` is the guard mask; ``s[k]``, ``f_re[k]``, ``f_im[k]`` belong to
    projection block ``k = 1..rounds`` (``f_re[0]``/``f_im[0]`` are unused).
    """
    s: List[np.ndarray]
    f_re: List[Optional[np.ndarray]]
    f_im: List[Optional[np.ndarray]]


@dataclasses.dataclass
class Result:
    y: np.ndarray                 # corrected data in the output dtype
    eps: np.ndarray               # final spatial error in FP64 (before output rounding)
    status: int
    rounds: int
    converged: bool
    viol: List[int]               # v_k of every check, k = 0..rounds
    s_clipped: List[int]          # spatial clips of every block (index 0: guard clip)
    margin: float
    max_spatial_err: float
    max_spectral_err: float
    masks: Optional[Masks] = None
    spat_edits: Optional[np.ndarray] = None   # sum of ProjectOntoSCube displacements (Alg. 1)
    freq_edits: Optional[np.ndarray] = None   # sum of ProjectOntoFCube displacements, half-spectrum


def _check_args(x, xb, E, Delta, max_iter):
    if x.shape != xb.shape:
        raise OracleError(E_SHAPE, "x and x_hat shapes differ")
    if x.ndim < 1 or x.ndim > 3 or any(n < 1 for n in x.shape):
        raise OracleError(E_SHAPE, "ndim must be 1..3 with every extent >= 1")
    for v, name in ((E, "E"), (Delta, "Delta")):
        if not math.isfinite(v) or v < 0.0:
            raise OracleError(E_INVALID, f"{name} must be finite and >= 0")
    if max_iter < 0:
        raise OracleError(E_INVALID, "max_iter must be >= 0")
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(xb))):
        raise OracleError(E_NONFINITE, "non-finite input")


def correct(x, xb, E: float, Delta: float, max_iter: int, *, mu: Optional[float] = None,
            fixed: bool = False, record_masks: bool = False, out_dtype=None,
            verify_output: bool = True, progress=None, record_edits: bool = False,
            thresholds: Optional[tuple] = None) -> Result:
    """Alg. 1 (alternating projection-correction), FP64 throughout.

    ``x``: original data, ``xb``: base-compressor reconstruction (same shape),
    ``E``: spatial bound, ``Delta``: bound on Re and Im of every frequency error,
    ``max_iter``: cap on projection blocks.  ``fixed``: run exactly ``max_iter``
    blocks regardless of the check (used for differentiation).
    ``out_dtype``: dtype of ``y`` (default: the dtype of ``x``).
    ``progress``: optional callable ``(k, v_k)`` invoked after each check (no effect on results).
    ``record_edits``: keep the edit bookkeeping of Alg. 1 -- ``spat_edits`` sums every
    displacement ``eps' - eps`` of ProjectOntoSCube (the guard clip included) and
    ``freq_edits`` every ``delta' - delta`` of ProjectOntoFCube (half-spectrum), so that
    ``eps_final = (x_hat - x) + spat_edits + IFFT(freq_edits)``.
    ``thresholds``: ``(E_p, Delta_c, Delta_p)`` overriding the ones derived from ``mu``.
    """
    x = np.asarray(x)
    xb = np.asarray(xb)
    _check_args(x, xb, float(E), float(Delta), int(max_iter))
    out_dtype = np.dtype(out_dtype if out_dtype is not None else x.dtype)
    if mu is None:
        mu = DEFAULT_MU if out_dtype == np.float64 else suggest_margin(x, Delta)
    shape = x.shape
    x64 = x.astype(np.float64)
    if thresholds is None:
        Ep = E * (1.0 - mu)
        Dc, Dp = spectral_thresholds(Delta, mu, out_dtype)
    else:
        Ep, Dc, Dp = (float(v) for v in thresholds)

    # Alg. 1, first statement: the spatial error of the base reconstruction.
    eps_raw = xb.astype(np.float64) - x64
    # Guard: the method starts inside the s-cube (Sec. IV-B).
    eps, keep, n_guard = project_s(eps_raw, Ep)
    masks = Masks([keep], [None], [None]) if record_masks else None
    # edit bookkeeping (Alg. 1): the guard clip is the first ProjectOntoSCube displacement
    spat_edits = (eps - eps_raw) if record_edits else None
    freq_edits = None

    viol: List[int] = []
    s_clipped = [n_guard]
    k = 0
    converged = False
    while True:
        delta = fft(eps)                          # FFT
        v = count_violations(delta, Dc)           # CheckConvergence
        viol.append(v)
        if progress is not None:
            progress(k, v)
        if v == 0 and not fixed:
            converged = True
            break
        if k == max_iter:
            converged = v == 0
            break
        delta_p, kre, kim = project_f(delta, Dp)  # ProjectOntoFCube
        if record_edits:
            d = delta_p - delta                   # freq_edits += delta' - delta
            freq_edits = d if freq_edits is None else freq_edits + d
        eps_pre = ifft(delta_p, shape)            # IFFT
        eps, ks, ns = project_s(eps_pre, Ep)      # ProjectOntoSCube
        if record_edits:
            spat_edits = spat_edits + (eps - eps_pre)  # spat_edits += eps' - eps
        s_clipped.append(ns)
        if masks is not None:
            masks.s.append(ks)
            masks.f_re.append(kre)
            masks.f_im.append(kim)
        k += 1

    y64 = x64 + eps
    if out_dtype == np.float64:
        y = y64
    else:
        y = closing_clamp(y64.astype(out_dtype), x, E)

    status = OK if converged or fixed else NOT_CONVERGED
    ms = mf = float("nan")
    if verify_output:
        ms, mf, _, ok = verify(x, y, E, Delta)
        if not ok and status == OK:
            status = VERIFY_FAILED
    if record_edits and freq_edits is None:
        freq_edits = np.zeros(fft(np.zeros(shape)).shape, dtype=np.complex128)
    return Result(y=y, eps=eps, status=status, rounds=k, converged=converged,
                  viol=viol, s_clipped=s_clipped, margin=float(mu),
                  max_spatial_err=ms, max_spectral_err=mf, masks=masks,
                  spat_edits=spat_edits, freq_edits=freq_edits)


def apply_f_mask(G: np.ndarray, keep_re: np.ndarray, keep_im: np.ndarray) -> np.ndarray:
    """Derivative of ProjectOntoFCube with frozen masks: keep Re and Im where unclipped."""
    return np.where(keep_re, G.real, 0.0) + 1j * np.where(keep_im, G.imag, 0.0)


def adjoint(masks: Masks, grad_y: np.ndarray) -> np.ndarray:
    """Vector-Jacobian product of the fixed-round map ``x_hat -> y``.

    Round ``k`` maps ``eps -> M_s^k (F^-1 M_f^k F eps)`` (clips replaced by their
    masks).  ``F^-1 M_f F`` is symmetric because the cos/sin vectors are
    orthogonal (Sec. IV-A), so the transpose of the whole trajectory applies the
    same factors in reverse order, ending with the guard mask.  The output clamp
    is treated as the identity.
    """
    shape = grad_y.shape
    K = len(masks.s) - 1
    g = np.asarray(grad_y, dtype=np.float64) * masks.s[K]
    for k in range(K, 0, -1):
        G = fft(g)
        G = apply_f_mask(G, masks.f_re[k], masks.f_im[k])
        g = ifft(G, shape)
        g = g * masks.s[k - 1]
    return g


def forward_fixed_masks(masks: Masks, v: np.ndarray) -> np.ndarray:
    """Jacobian-vector product of the same map (masks frozen), forward order."""
    shape = v.shape
    K = len(masks.s) - 1
    g = np.asarray(v, dtype=np.float64) * masks.s[0]
    for k in range(1, K + 1):
        G = apply_f_mask(fft(g), masks.f_re[k], masks.f_im[k])
        g = ifft(G, shape) * masks.s[k]
    return g


def default_workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
