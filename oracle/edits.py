"""FP64 CPU oracle of the edit coding around the correction loop (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

What is computed (paper Alg. 1, Sec. IV-B "Compaction, quantization, and lossless
compression of edits" and "Applying edits to the decompressed data", Sec. IV-D):

* edit bookkeeping: the loop sums every ProjectOntoSCube displacement into
  ``spat_edits`` and every ProjectOntoFCube displacement into ``freq_edits``
  (``oracle.ffcz.correct(record_edits=True)``);
* CompactEdits: a flag per coordinate (set iff the edit is non-zero), packed
  eight to a byte, and the non-zero edits in coordinate order, each placed at the
  exclusive prefix count of the flags before it;
* QuantizeEdits: each axis of the s-cube (``[-E, E]``) or f-cube (``[-Delta,
  Delta]``) is cut into ``2^m`` intervals, so an edit ``v`` becomes the integer
  ``rint(v / step)`` with ``step = 2 bound 2^-m``;
* decoding: ``y = x_hat + spatial edits + IFFT(frequency edits)`` from the
  dequantised codes.

Readings taken where the paper is silent:

* Coordinates.  Spatial: the N field values in C order.  Frequency: the Re and Im
  parts of every half-spectrum entry (the entries of ``rfftn``, C order), Re before
  Im -- the frequency basis of Sec. IV-A, one coordinate per cos or sin vector
  (the Im coordinates of self-conjugate entries never carry an edit).
* Flag bytes hold coordinates ``8b .. 8b+7`` in bits 0..7 (least significant bit
  first); a final partial byte is zero-padded.
* Codes are signed integers (int32): an accumulated edit is not confined to one
  cube side, so ``m`` fixes the step, not the code range.  ``rint`` rounds half to even.
* The guard clip that puts the initial error inside the s-cube is the first
  ProjectOntoSCube displacement and is recorded as a spatial edit, so decoding
  reproduces it.
* Shrink.  The paper shrinks both bounds by ``2^-m`` so that the quantised edits
  still land inside.  That argument counts each edit's own rounding only: the
  quantisation error of one domain also reaches the other through the transform,
  and an FP32 decoder rounds its output with no closing clamp (it does not know
  ``x``).  The encoder therefore runs the loop with the check at
  ``Delta (1 - mu_f)``, the f-projection at ``Delta (1 - 2 mu_f)`` and the
  s-projection at ``E (1 - mu_s)``, where ``mu_f = max(mu_out, safety 2^-m)``
  (``mu_out``: the output-rounding margin of the plain correction) and
  ``mu_s = safety 2^-m + ulp(max|x| + E) / E`` (a whole output ulp, twice the
  rounding error); ``safety = 4`` by default, and the decoded output is
  re-verified in FP64 instead of trusted.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from oracle import ffcz as O

DEFAULT_M = 16       # code length m (Sec. IV-B fixes m = 16)
DEFAULT_SAFETY = 4.0  # shrink in units of 2^-m (the paper's own argument uses 1)


# ----------------------------------------------------------------------------- coordinates

def spatial_coords(spat_edits: np.ndarray) -> np.ndarray:
    """Spatial edits as a flat FP64 vector of N coordinates (C order)."""
    return np.ascontiguousarray(spat_edits, dtype=np.float64).reshape(-1)


def freq_coords(freq_edits: np.ndarray) -> np.ndarray:
    """Half-spectrum edits as 2M real coordinates: Re, Im of each entry in C order."""
    f = np.ascontiguousarray(freq_edits, dtype=np.complex128)
    return np.stack([f.real, f.imag], axis=-1).reshape(-1)


def freq_from_coords(c: np.ndarray, hshape) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64).reshape(tuple(hshape) + (2,))
    return c[..., 0] + 1j * c[..., 1]


# ----------------------------------------------------------------------------- CompactEdits

def compact(values: np.ndarray):
    """CompactEdits (Alg. 1; Sec. IV-D): flags packed eight per byte (LSB first)
    and the non-zero values in coordinate order (positions = exclusive prefix count)."""
    v = np.asarray(values, dtype=np.float64).reshape(-1)
    nz = v != 0.0
    flags = np.packbits(nz, bitorder="little")
    return flags, v[nz].copy()


def expand(flags: np.ndarray, compact_values: np.ndarray, n: int) -> np.ndarray:
    """Inverse of ``compact``: dense vector of ``n`` coordinates (zeros where unflagged)."""
    bits = np.unpackbits(np.asarray(flags, dtype=np.uint8), bitorder="little")[:n].astype(bool)
    out = np.zeros(n, dtype=np.asarray(compact_values).dtype if np.asarray(compact_values).size else np.float64)
    if int(bits.sum()) != np.asarray(compact_values).size:
        raise ValueError("flag count and compact length differ")
    out[bits] = compact_values
    return out


# ----------------------------------------------------------------------------- QuantizeEdits

def step(bound: float, m: int = DEFAULT_M) -> float:
    """Quantisation step: one of the 2^m intervals of a cube side ``[-bound, bound]``."""
    return 2.0 * float(bound) * 2.0 ** (-int(m))


def quantize(values: np.ndarray, st: float) -> np.ndarray:
    """QuantizeEdits (Alg. 1; Sec. IV-B): ``rint(v / step)`` as int32 (half to even)."""
    v = np.asarray(values, dtype=np.float64)
    if st <= 0.0:
        if np.any(v != 0.0):
            raise ValueError("a zero step quantises only zeros")
        return np.zeros(v.shape, dtype=np.int32)
    q = np.rint(v / st)
    if q.size and float(np.max(np.abs(q))) >= 2.0 ** 31:
        raise OverflowError("edit beyond the int32 code range")
    return q.astype(np.int32)


def dequantize(codes: np.ndarray, st: float) -> np.ndarray:
    return np.asarray(codes, dtype=np.float64) * float(st)


# ----------------------------------------------------------------------------- margins

def encode_margins(x: np.ndarray, E: float, Delta: float, out_dtype, m: int = DEFAULT_M,
                   safety: float = DEFAULT_SAFETY):
    """``(mu_s, mu_f)`` of the encoder (see the module docstring)."""
    out_dtype = np.dtype(out_dtype)
    q = float(safety) * 2.0 ** (-int(m))
    mu_out = O.DEFAULT_MU if out_dtype == np.float64 else O.suggest_margin(x, Delta)
    mu_f = max(mu_out, q)
    xm = float(np.max(np.abs(np.asarray(x, dtype=np.float64)))) if np.asarray(x).size else 0.0
    u = float(np.spacing(out_dtype.type(xm + E))) if E > 0 else 0.0
    mu_s = q + (u / E if E > 0 else 0.0)
    return float(min(mu_s, 0.5)), float(min(mu_f, 0.25))


def encode_thresholds(E: float, Delta: float, mu_s: float, mu_f: float):
    """``(E_p, Delta_c, Delta_p)``: s-projection bound, check bound, f-projection bound."""
    return E * (1.0 - mu_s), Delta * (1.0 - mu_f), Delta * (1.0 - 2.0 * mu_f)


# ----------------------------------------------------------------------------- encoder / decoder

@dataclasses.dataclass
class Encoded:
    shape: tuple
    spat_flags: np.ndarray     # uint8, ceil(N / 8)
    spat_codes: np.ndarray     # int32, nnz_s
    freq_flags: np.ndarray     # uint8, ceil(2M / 8)
    freq_codes: np.ndarray     # int32, nnz_f
    step_s: float
    step_f: float
    rounds: int
    converged: bool
    mu_s: float
    mu_f: float
    spat_edits: np.ndarray     # FP64 accumulators before coding (for checks)
    freq_edits: np.ndarray
    eps: np.ndarray            # final error of the loop (FP64)


def encode(x, xb, E: float, Delta: float, max_iter: int, *, m: int = DEFAULT_M,
           safety: float = DEFAULT_SAFETY, out_dtype=None, mus: Optional[tuple] = None) -> Encoded:
    """Alg. 1 end to end: the loop with edit bookkeeping, CompactEdits and QuantizeEdits
    on both domains (lossless coding aside)."""
    x = np.asarray(x)
    out_dtype = np.dtype(out_dtype if out_dtype is not None else x.dtype)
    mu_s, mu_f = mus if mus is not None else encode_margins(x, E, Delta, out_dtype, m, safety)
    thr = encode_thresholds(E, Delta, mu_s, mu_f)
    r = O.correct(x, xb, E, Delta, max_iter, mu=mu_f, out_dtype=out_dtype, verify_output=False,
                  record_edits=True, thresholds=thr)
    ss, sf = step(E, m), step(Delta, m)
    fs, vs = compact(spatial_coords(r.spat_edits))
    ff, vf = compact(freq_coords(r.freq_edits))
    return Encoded(shape=tuple(x.shape), spat_flags=fs, spat_codes=quantize(vs, ss), freq_flags=ff,
                   freq_codes=quantize(vf, sf), step_s=ss, step_f=sf, rounds=r.rounds,
                   converged=r.converged, mu_s=mu_s, mu_f=mu_f, spat_edits=r.spat_edits,
                   freq_edits=r.freq_edits, eps=r.eps)


def half_shape(shape) -> tuple:
    shape = tuple(shape)
    return shape[:-1] + (shape[-1] // 2 + 1,)


def decode_edits(enc: Encoded):
    """Dense dequantised edits ``(spatial FP64 field, half-spectrum complex)``."""
    n = int(np.prod(enc.shape))
    hs = half_shape(enc.shape)
    s = expand(enc.spat_flags, dequantize(enc.spat_codes, enc.step_s), n).reshape(enc.shape)
    f = freq_from_coords(expand(enc.freq_flags, dequantize(enc.freq_codes, enc.step_f), 2 * int(np.prod(hs))), hs)
    return s, f


def decode(xb, enc: Encoded, out_dtype=None) -> np.ndarray:
    """Applying edits (Sec. IV-B): ``y = x_hat + s + IFFT(f)`` in FP64, rounded once to the dtype."""
    xb = np.asarray(xb)
    out_dtype = np.dtype(out_dtype if out_dtype is not None else xb.dtype)
    s, f = decode_edits(enc)
    y64 = xb.astype(np.float64) + s + O.ifft(f, enc.shape)
    return y64.astype(out_dtype)
