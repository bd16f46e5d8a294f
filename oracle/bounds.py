"""FP64 CPU oracle of the generalised bounds (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

What is computed
----------------
* Pointwise bounds (the footnote to Eq. 2, Sec. IV-A): ``|eps_n| <= E_n`` for
  every point and ``|Re delta_k| <= D^Re_k``, ``|Im delta_k| <= D^Im_k`` for every
  half-spectrum entry.  The loop is Alg. 1 with every clip taken against its own
  entry's bound.
* The disk variant ``|delta_k| <= D_k``: the modulus, the quantity the relative
  frequency error of Sec. V measures (Eq. 2 itself is a box on Re and Im).  Its
  projection scales an outside coefficient radially onto the circle.
* Relative power-spectrum bounds (Sec. V-B, Observation 4: a relative bound on
  every power-spectrum component, reached through pointwise frequency bounds):
  a relative bound ``rho`` on every shell ``P(b)`` of the power spectrum
  (Sec. III) becomes one ``D_b`` for all entries of shell ``b``.

Readings taken where the paper is silent
----------------------------------------
* Thresholds per entry as in the scalar oracle: FP64 output -- check against
  ``D_k``, project onto ``E_n (1 - mu)``, ``D_k (1 - mu)``; FP32 output -- check
  against ``D_k (1 - mu)``, project onto ``D_k (1 - 2 mu)``.  The FP32 output
  margin is the scalar rule with ``Delta = min_k D_k`` (the rounding noise of
  the output is the same at every k, so the smallest bound sets the relative
  margin); for the disk it is multiplied by ``sqrt 2`` (noise in both parts).
* A half-spectrum bound array defines the full-spectrum bound by Hermitian
  symmetry (``D_{-k} = D_k``), so clipping the half-spectrum equals clipping the
  full spectrum; the Im bound of a self-conjugate entry never acts.
* Shells: ``b = rint(|k|)`` with ``|k|`` from the signed integer frequencies
  (the binning of ``oracle.spectrum``), every shell from ``b = 0`` (DC) up, with
  the full-spectrum weights ``w_k`` (2 for interior last-axis entries, 1 at
  ``k_z = 0`` and at the Nyquist plane of an even last axis).
* Per-shell bound.  For an error inside the bounds,
  ``|P_hat(b) - P(b)| = |sum_k w_k (2 Re(conj(X_k) delta_k) + |delta_k|^2)|``
  is at most ``sum_k w_k (2 |X_k| r + r^2)`` with ``r`` the largest ``|delta_k|``
  the bound allows (``sqrt 2 D`` for the box, ``D`` for the disk).  With
  ``S_b = sum w_k |X_k|`` and ``W_b = sum w_k`` the largest ``D_b`` keeping that
  below ``rho P(b)`` is the positive root of a quadratic:
  box ``D_b = (sqrt(2 S_b^2 + 2 W_b rho P(b)) - sqrt 2 S_b) / (2 W_b)``,
  disk ``D_b = (sqrt(S_b^2 + W_b rho P(b)) - S_b) / W_b``, evaluated as
  ``rho P(b) / (sqrt(...) + sqrt 2 S_b)`` and ``rho P(b) / (sqrt(...) + S_b)`` (no
  cancellation; 0 for a shell of zero power).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from oracle import ffcz as O


def half_shape(shape) -> tuple:
    shape = tuple(int(n) for n in shape)
    return shape[:-1] + (shape[-1] // 2 + 1,)


def as_spatial(E, shape) -> np.ndarray:
    """Spatial bounds as an FP64 array of the field's shape (a scalar is broadcast)."""
    return np.broadcast_to(np.asarray(E, dtype=np.float64), tuple(shape)).copy()


def as_spectral(D, shape) -> np.ndarray:
    """Spectral bounds as an FP64 array of the half-spectrum shape (a scalar is broadcast)."""
    return np.broadcast_to(np.asarray(D, dtype=np.float64), half_shape(shape)).copy()


# ----------------------------------------------------------------------------- projections

def project_s(eps: np.ndarray, Ep: np.ndarray):
    """ProjectOntoSCube with a bound per point: clip ``eps_n`` to ``[-Ep_n, Ep_n]``."""
    keep = np.abs(eps) <= Ep
    out = np.where(eps > Ep, Ep, np.where(eps < -Ep, -Ep, eps))
    return out, keep, int(eps.size - np.count_nonzero(keep))


def project_f_box(delta: np.ndarray, Dp_re: np.ndarray, Dp_im: np.ndarray):
    """ProjectOntoFCube with a bound per entry and part: clip Re to ``[-Dp_re, Dp_re]``
    and Im to ``[-Dp_im, Dp_im]``."""
    re, im = delta.real, delta.imag
    keep_re = np.abs(re) <= Dp_re
    keep_im = np.abs(im) <= Dp_im
    re2 = np.where(re > Dp_re, Dp_re, np.where(re < -Dp_re, -Dp_re, re))
    im2 = np.where(im > Dp_im, Dp_im, np.where(im < -Dp_im, -Dp_im, im))
    return re2 + 1j * im2, keep_re, keep_im


def project_f_disk(delta: np.ndarray, Dp: np.ndarray):
    """Projection onto the disks ``|delta_k| <= Dp_k``: a coefficient outside its disk
    moves radially onto the circle, ``delta Dp / |delta|``; the rest are kept."""
    mag = np.abs(delta)
    keep = mag <= Dp
    with np.errstate(divide="ignore", invalid="ignore"):
        scaled = delta * (Dp / mag)
    return np.where(keep, delta, scaled), keep


def count_box(delta: np.ndarray, Dc_re: np.ndarray, Dc_im: np.ndarray) -> int:
    bad = (np.abs(delta.real) > Dc_re) | (np.abs(delta.imag) > Dc_im)
    return int(np.count_nonzero(bad))


def count_disk(delta: np.ndarray, Dc: np.ndarray) -> int:
    return int(np.count_nonzero(np.abs(delta) > Dc))


# ----------------------------------------------------------------------------- margin

def suggest_margin(x: np.ndarray, D_min: float, disk: bool = False) -> float:
    """FP32 output margin of the scalar oracle with ``Delta = min_k D_k`` (times sqrt 2 for
    the disk), at least 2^-16 and at most 1/2."""
    x = np.asarray(x)
    u = O.ulp32(x)
    sigma = math.sqrt(float(np.mean(u * u)) / 12.0)
    if D_min <= 0.0:
        return 0.5
    mu = 8.0 * sigma * math.sqrt(x.size / 2.0) / D_min
    if disk:
        mu *= math.sqrt(2.0)
    return float(min(0.5, max(O.DEFAULT_MU, mu)))


# ----------------------------------------------------------------------------- the loop

@dataclasses.dataclass
class Result:
    y: np.ndarray
    eps: np.ndarray
    status: int
    rounds: int
    converged: bool
    viol: List[int]
    s_clipped: List[int]
    margin: float


def correct(x, xb, E, D_re, max_iter: int, *, D_im=None, disk: bool = False, mu: Optional[float] = None,
            fixed: bool = False, out_dtype=None) -> Result:
    """Alg. 1 with pointwise bounds (arrays or scalars broadcast to them), FP64 throughout.

    ``E``: spatial bounds (field shape); ``D_re`` / ``D_im``: spectral bounds on Re / Im
    (half-spectrum shape; ``D_im`` defaults to ``D_re``); ``disk``: bound the modulus by
    ``D_re`` instead.  The FP32 closing clamp moves each output toward x until
    ``|y_n - x_n| <= E_n``.
    """
    x = np.asarray(x)
    xb = np.asarray(xb)
    shape = x.shape
    out_dtype = np.dtype(out_dtype if out_dtype is not None else x.dtype)
    E = as_spatial(E, shape)
    D_re = as_spectral(D_re, shape)
    D_im = D_re if (D_im is None or disk) else as_spectral(D_im, shape)
    if max_iter < 0 or np.any(E < 0) or np.any(D_re < 0) or np.any(D_im < 0):
        raise O.OracleError(O.E_INVALID, "bounds must be >= 0 and max_iter >= 0")
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(xb))):
        raise O.OracleError(O.E_NONFINITE, "non-finite input")
    dmin = float(min(D_re.min(), D_im.min())) if D_re.size else 0.0
    if mu is None:
        mu = O.DEFAULT_MU if out_dtype == np.float64 else suggest_margin(x, dmin, disk)
    rho = 0.0 if out_dtype == np.float64 else mu
    Ep = E * (1.0 - mu)
    Dc_re, Dp_re = D_re * (1.0 - rho), D_re * (1.0 - rho - mu)
    Dc_im, Dp_im = D_im * (1.0 - rho), D_im * (1.0 - rho - mu)

    x64 = x.astype(np.float64)
    eps, _, n_guard = project_s(xb.astype(np.float64) - x64, Ep)   # guard clip
    viol, s_clipped = [], [n_guard]
    k = 0
    converged = False
    while True:
        delta = O.fft(eps)
        v = count_disk(delta, Dc_re) if disk else count_box(delta, Dc_re, Dc_im)
        viol.append(v)
        if v == 0 and not fixed:
            converged = True
            break
        if k == max_iter:
            converged = v == 0
            break
        if disk:
            delta, _ = project_f_disk(delta, Dp_re)
        else:
            delta, _, _ = project_f_box(delta, Dp_re, Dp_im)
        eps, _, ns = project_s(O.ifft(delta, shape), Ep)
        s_clipped.append(ns)
        k += 1
    y64 = x64 + eps
    if out_dtype == np.float64:
        y = y64
    else:
        y = closing_clamp(y64.astype(out_dtype), x, E)
    status = O.OK if converged or fixed else O.NOT_CONVERGED
    return Result(y=y, eps=eps, status=status, rounds=k, converged=converged, viol=viol,
                  s_clipped=s_clipped, margin=float(mu))


def closing_clamp(y32: np.ndarray, x: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Move each FP32 output one ulp at a time toward x until ``|y_n - x_n| <= E_n`` in FP64."""
    y32 = np.array(y32, dtype=np.float32, copy=True)
    x64 = np.asarray(x, dtype=np.float64)
    xs = np.asarray(x, dtype=np.float32)
    bad = np.abs(y32.astype(np.float64) - x64) > E
    while np.any(bad):
        idx = np.nonzero(bad)
        y32[idx] = np.nextafter(y32[idx], xs[idx])
        bad = np.abs(y32.astype(np.float64) - x64) > E
    return y32


def verify(x, y, E, D_re, D_im=None, disk: bool = False):
    """FP64 re-verification against pointwise bounds.  Returns ``(max |d_n| / E_n,
    max spectral ratio, spectral violations, ok)``; the ratios take 0/0 as 0."""
    x = np.asarray(x)
    shape = x.shape
    E = as_spatial(E, shape)
    D_re = as_spectral(D_re, shape)
    D_im = D_re if (D_im is None or disk) else as_spectral(D_im, shape)
    d = np.asarray(y, dtype=np.float64) - np.asarray(x, dtype=np.float64)
    Dk = O.fft(d)

    def ratio(a, b):
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(a == 0, 0.0, a / b)
        return float(np.max(r)) if r.size else 0.0

    rs = ratio(np.abs(d), E)
    if disk:
        rf = ratio(np.abs(Dk), D_re)
        nv = count_disk(Dk, D_re)
    else:
        rf = max(ratio(np.abs(Dk.real), D_re), ratio(np.abs(Dk.imag), D_im))
        nv = count_box(Dk, D_re, D_im)
    ok = bool(np.all(np.abs(d) <= E)) and nv == 0
    return rs, rf, nv, ok


# ----------------------------------------------------------------------------- power spectrum

def shells(shape):
    """Shell index ``rint(|k|)`` and full-spectrum weight of every half-spectrum entry."""
    shape = tuple(int(n) for n in shape)
    axes = []
    for i, n in enumerate(shape):
        f = np.arange(n // 2 + 1, dtype=np.float64) if i == len(shape) - 1 else np.fft.fftfreq(n) * n
        axes.append(f)
    grids = np.meshgrid(*axes, indexing="ij")
    b = np.rint(np.sqrt(sum(g * g for g in grids))).astype(np.int64)
    nl = shape[-1]
    kz = np.arange(nl // 2 + 1)
    w1 = np.where((kz == 0) | ((nl % 2 == 0) & (kz == nl // 2)), 1.0, 2.0)
    return b, np.broadcast_to(w1, b.shape).astype(np.float64)


def shell_power(X: np.ndarray, b: np.ndarray, w: np.ndarray) -> np.ndarray:
    """``P(b) = sum_{k in shell b} w_k |X_k|^2`` for every shell b = 0 .. max."""
    return np.bincount(b.ravel(), weights=(w * np.abs(X) ** 2).ravel(), minlength=int(b.max()) + 1)


def power_spectrum_bounds(x, rho: float, disk: bool = False) -> np.ndarray:
    """Pointwise spectral bound (half-spectrum shape) that keeps every shell of the power
    spectrum within ``rho`` relative error: one ``D_b`` per shell, see the module docstring."""
    x = np.asarray(x, dtype=np.float64)
    X = O.fft(x)
    b, w = shells(x.shape)
    nb = int(b.max()) + 1
    P = np.bincount(b.ravel(), weights=(w * np.abs(X) ** 2).ravel(), minlength=nb)
    S = np.bincount(b.ravel(), weights=(w * np.abs(X)).ravel(), minlength=nb)
    Wt = np.bincount(b.ravel(), weights=w.ravel(), minlength=nb)
    # the positive root of the quadratic, in the form without cancellation:
    # disk (sqrt(S^2 + W rho P) - S) / W = rho P / (sqrt(S^2 + W rho P) + S), box likewise
    if disk:
        den = np.sqrt(S * S + Wt * rho * P) + S
    else:
        den = np.sqrt(2.0 * S * S + 2.0 * Wt * rho * P) + math.sqrt(2.0) * S
    with np.errstate(divide="ignore", invalid="ignore"):
        Db = np.where(den > 0, rho * P / den, 0.0)
    return Db[b]
