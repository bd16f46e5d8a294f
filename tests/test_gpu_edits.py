"""Edit coding on the GPU against the oracle (Alg. 1 edit bookkeeping, CompactEdits and
QuantizeEdits, Sec. IV-B / IV-D; applying edits, Sec. IV-B), through the C ABI.

- CompactEdits + QuantizeEdits: the oracle's compaction and quantiser applied to the
  GPU's own accumulators give the GPU's flags and codes bit for bit (same values, same
  decision in FP64).
- Edit bookkeeping: the GPU's accumulators against the oracle loop with the same shrinks
  (FP64: same flags, values to 1e-10 of the bounds; FP32: values to 1e-4 of the bounds).
- FP64 end to end: flags identical to the oracle encoder's, codes identical except where
  the oracle's value sits within 1e-6 of a rounding tie.
- Decoder: against the oracle decoder on the same flags and codes; the decoded output meets
  both bounds in FP64 and lies within the quantisation bound of the encoder's own y.
- Full size: the 512^3 FP32 lognormal field (the benchmark workload) encoded, its codes
  checked against the oracle's coding of its accumulators, decoded and re-verified.
"""

import numpy as np
import pytest

from oracle import edits as ED
from oracle import ffcz as O
from paper_2601_01596_amd import ffcz as F
from paper_2601_01596_amd import workloads as W
from tests.progress import say

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    return t.cpu().numpy()


def _problem(kind, dt):
    if kind == "grf64":
        p = W.config_grf_fp64(64)
        return p.x.astype(dt), W.quantize(p.x, p.E).astype(dt), p.E, p.Delta, 200
    if kind == "lognormal32":
        p = W.config_lognormal(32, dt)
        return p.x, p.xb, p.E, p.Delta, 200
    if kind == "hedm256":
        p = W.config_diffraction(7, 256)
        x = p.x.astype(dt)
        xb = W.quantize(x, p.E).astype(dt)
        return x, xb, p.E, W.spectral_bound(x, xb, 90.0), 200
    if kind == "eeg4096":
        x = W.eeg_signal(3, 4096).astype(dt)
        E = W.spatial_bound(x, 1e-3)
        xb = W.quantize(x, E).astype(dt)
        return x, xb, E, W.spectral_bound(x, xb, 90.0), 200
    if kind == "ragged":  # a 3D field with few rows per plane and a short last axis
        g = np.random.default_rng(77)
        x = W.grf((16, 8, 32), 2.0, 9).astype(dt)
        E = W.spatial_bound(x, 2e-2)
        xb = W.quantize(x, E).astype(dt)
        return x, xb, E, W.spectral_bound(x, xb, 85.0), 300
    raise KeyError(kind)


def _oracle_encoded(enc):
    """The GPU's flags and codes as an oracle ``Encoded`` (for the oracle decoder)."""
    return ED.Encoded(shape=tuple(enc.shape), spat_flags=_np(enc.spat_flags), spat_codes=_np(enc.spat_codes),
                      freq_flags=_np(enc.freq_flags), freq_codes=_np(enc.freq_codes), step_s=enc.step_s,
                      step_f=enc.step_f, rounds=enc.stats["rounds"], converged=bool(enc.stats["converged"]),
                      mu_s=enc.mu_s, mu_f=enc.mu_f, spat_edits=None, freq_edits=None, eps=None)


CASES = [("grf64", np.float64), ("grf64", np.float32), ("lognormal32", np.float32), ("lognormal32", np.float64),
         ("hedm256", np.float32), ("eeg4096", np.float32), ("eeg4096", np.float64), ("ragged", np.float64),
         ("ragged", np.float32)]


@pytest.mark.parametrize("kind,dt", CASES)
def test_coding_kernels_reproduce_the_oracle_coding_of_the_accumulators(kind, dt):
    x, xb, E, D, K = _problem(kind, dt)
    enc = F.encode(_dev(x), _dev(xb), E, D, K, export_edits=True)
    assert enc.status == F.OK, (enc.status, F.ffcz_last_error())
    se, fe = _np(enc.spat_edits).astype(np.float64), _np(enc.freq_edits).astype(np.float64)
    fs, vs = ED.compact(se)
    ff, vf = ED.compact(fe)
    np.testing.assert_array_equal(_np(enc.spat_flags), fs)
    np.testing.assert_array_equal(_np(enc.freq_flags), ff)
    np.testing.assert_array_equal(_np(enc.spat_codes), ED.quantize(vs, enc.step_s))
    np.testing.assert_array_equal(_np(enc.freq_codes), ED.quantize(vf, enc.step_f))
    assert enc.step_s == ED.step(E) and enc.step_f == ED.step(D)
    say(f"[edits] {kind} {np.dtype(dt).name}: rounds {enc.stats['rounds']}, nnz_s {vs.size}, nnz_f {vf.size}")


@pytest.mark.parametrize("kind,dt", CASES)
def test_accumulators_and_shrinks_match_the_oracle(kind, dt):
    x, xb, E, D, K = _problem(kind, dt)
    enc = F.encode(_dev(x), _dev(xb), E, D, K, export_edits=True)
    assert enc.status == F.OK, (enc.status, F.ffcz_last_error())
    # the shrinks derived on the device are the oracle's (FP32 output margin: summation order)
    ms, mf = ED.encode_margins(x, E, D, dt)
    assert enc.mu_s == ms
    assert enc.mu_f == pytest.approx(mf, rel=1e-12)
    thr = ED.encode_thresholds(E, D, enc.mu_s, enc.mu_f)
    r = O.correct(x, xb, E, D, K, mu=enc.mu_f, out_dtype=dt, verify_output=False, record_edits=True,
                  thresholds=thr)
    k = enc.stats["rounds"]
    if k != r.rounds:
        assert dt == np.float32 and abs(k - r.rounds) <= 1
        r = O.correct(x, xb, E, D, k, mu=enc.mu_f, out_dtype=dt, verify_output=False, record_edits=True,
                      thresholds=thr, fixed=True)
    se = _np(enc.spat_edits).astype(np.float64)
    fe = _np(enc.freq_edits).astype(np.float64)
    so = ED.spatial_coords(r.spat_edits)
    fo = ED.freq_coords(r.freq_edits)
    es = float(np.max(np.abs(se - so))) / E
    ef = float(np.max(np.abs(fe - fo))) / D
    say(f"[edits] {kind} {np.dtype(dt).name}: |s - s_orc| {es:.2e} E, |f - f_orc| {ef:.2e} Delta")
    if dt == np.float64:
        assert k == r.rounds
        np.testing.assert_array_equal(se != 0, so != 0)
        np.testing.assert_array_equal(fe != 0, fo != 0)
        assert es <= 1e-10 and ef <= 1e-10
    else:
        assert es <= 1e-4 and ef <= 1e-4
        # a flag differs only where the two precisions decide a clip at its bound
        assert np.count_nonzero((se != 0) != (so != 0)) <= 1e-3 * se.size + 2
        assert np.count_nonzero((fe != 0) != (fo != 0)) <= 1e-3 * fe.size + 2


@pytest.mark.parametrize("kind", ["grf64", "lognormal32", "eeg4096", "ragged", "hedm256"])
def test_fp64_codes_match_the_oracle_encoder(kind):
    x, xb, E, D, K = _problem(kind, np.float64)
    enc = F.encode(_dev(x), _dev(xb), E, D, K)
    assert enc.status == F.OK
    orc = ED.encode(x, xb, E, D, K, mus=(enc.mu_s, enc.mu_f))
    assert orc.rounds == enc.stats["rounds"]
    np.testing.assert_array_equal(_np(enc.spat_flags), orc.spat_flags)
    np.testing.assert_array_equal(_np(enc.freq_flags), orc.freq_flags)
    for g, o, v, st in ((_np(enc.spat_codes), orc.spat_codes, ED.compact(ED.spatial_coords(orc.spat_edits))[1],
                         enc.step_s),
                        (_np(enc.freq_codes), orc.freq_codes, ED.compact(ED.freq_coords(orc.freq_edits))[1],
                         enc.step_f)):
        assert g.shape == o.shape
        bad = g != o
        if np.any(bad):
            frac = np.abs(np.abs(v[bad] / st - np.floor(v[bad] / st)) - 0.5)
            assert np.all(frac < 1e-6) and np.all(np.abs(g[bad] - o[bad]) == 1)


@pytest.mark.parametrize("kind,dt", CASES)
def test_decoder_matches_the_oracle_decoder_and_meets_both_bounds(kind, dt):
    x, xb, E, D, K = _problem(kind, dt)
    xbt = _dev(xb)
    enc = F.encode(_dev(x), xbt, E, D, K, want_y=True)
    assert enc.status == F.OK, (enc.status, F.ffcz_last_error())
    y = _np(F.decode(xbt, enc))
    assert y.dtype == np.dtype(dt)
    y_orc = ED.decode(xb, _oracle_encoded(enc))
    rel = float(np.max(np.abs(y.astype(np.float64) - y_orc.astype(np.float64)))) / float(np.max(np.abs(y_orc)))
    assert rel <= (1e-12 if dt == np.float64 else 1e-5), rel
    ms, mf, nv, ok = O.verify(x, y, E, D)
    say(f"[decode] {kind} {np.dtype(dt).name}: vs oracle decoder {rel:.1e}; max|y-x| {ms / E:.6f} E, "
        f"max spectral {mf / D:.6f} Delta")
    assert ok and nv == 0
    # distance to the encoder's own corrected field: the dequantisation error, plus output rounding
    y_enc = _np(enc.y).astype(np.float64)
    N = x.size
    bound = enc.step_s / 2 + 2.0 * enc.freq_codes.numel() / N * enc.step_f / 2
    bound += 2 * float(np.spacing(np.dtype(dt).type(np.max(np.abs(x)) + E)))
    assert float(np.max(np.abs(y.astype(np.float64) - y_enc))) <= bound * (1 + 1e-9)


def test_regimes_and_empty_edit_sets():
    import torch
    g = np.random.default_rng(5)
    # s-cube inside the f-cube: no round, no edits, decoding returns x_hat
    shape = (8, 16, 32)
    x = g.standard_normal(shape)
    xb = x + g.uniform(-0.9e-1, 0.9e-1, shape)
    enc = F.encode(_dev(x), _dev(xb), 0.1, x.size * 0.1, 50)
    assert enc.status == F.OK and enc.stats["rounds"] == 0
    assert enc.spat_codes.numel() == 0 and enc.freq_codes.numel() == 0
    assert int(enc.spat_flags.sum()) == 0 and int(enc.freq_flags.sum()) == 0
    y = _np(F.decode(_dev(xb), enc))
    np.testing.assert_array_equal(y, xb)
    # f-cube inside the s-cube: one round, frequency edits only (guard clip aside, none here)
    xb = x + 0.99 * g.uniform(-1, 1, shape)
    enc = F.encode(_dev(x), _dev(xb), 1.0, 0.5, 50, export_edits=True)
    assert enc.status == F.OK and enc.stats["rounds"] == 1
    assert enc.spat_codes.numel() == 0
    orc = ED.encode(x, xb, 1.0, 0.5, 50, mus=(enc.mu_s, enc.mu_f))
    np.testing.assert_array_equal(_np(enc.freq_flags), orc.freq_flags)
    y = _np(F.decode(_dev(xb), enc))
    assert O.verify(x, y, 1.0, 0.5)[3]
    # the smallest fields: two points, 2 x 2, a 4-point line
    for shape in ((2,), (2, 2), (4,), (2, 2, 2)):
        x = g.standard_normal(shape)
        xb = x + g.uniform(-0.5, 0.5, shape)
        E, D = 0.3, 0.2
        enc = F.encode(_dev(x), _dev(xb), E, D, 100)
        assert enc.status == F.OK, shape
        orc = ED.encode(x, xb, E, D, 100, mus=(enc.mu_s, enc.mu_f))
        np.testing.assert_array_equal(_np(enc.spat_flags), orc.spat_flags)
        np.testing.assert_array_equal(_np(enc.freq_flags), orc.freq_flags)
        y = _np(F.decode(_dev(xb), enc))
        np.testing.assert_allclose(y, ED.decode(xb, orc), rtol=0, atol=1e-12)
        assert O.verify(x, y, E, D)[3], shape


def test_decoder_rejects_a_wrong_code_count():
    x, xb, E, D, K = _problem("lognormal32", np.float32)
    xbt = _dev(xb)
    enc = F.encode(_dev(x), xbt, E, D, K)
    assert enc.freq_codes.numel() > 0
    enc.freq_codes = enc.freq_codes[:-1].clone()
    with pytest.raises(F.FFCzError) as ei:
        F.decode(xbt, enc)
    assert ei.value.status == F.E_INVALID


@pytest.mark.timeout(600)
def test_lognormal512_encode_decode_full_size():
    import torch
    O.set_workers(max(1, min(16, O.default_workers())))
    say("[edits] lognormal 512^3 FP32: generating")
    p = W.config_lognormal(512, np.float32)
    x, xb = _dev(p.x), _dev(p.xb)
    say("[edits] encoding on the GPU")
    enc = F.encode(x, xb, p.E, p.Delta, p.max_iter, export_edits=True)
    assert enc.status == F.OK, (enc.status, F.ffcz_last_error())
    say(f"[edits] rounds {enc.stats['rounds']}, nnz_s {enc.spat_codes.numel()}, nnz_f {enc.freq_codes.numel()}; "
        f"oracle coding of the accumulators")
    se = _np(enc.spat_edits).astype(np.float64)
    fs, vs = ED.compact(se)
    del se
    np.testing.assert_array_equal(_np(enc.spat_flags), fs)
    np.testing.assert_array_equal(_np(enc.spat_codes), ED.quantize(vs, enc.step_s))
    fe = _np(enc.freq_edits).astype(np.float64)
    ff, vf = ED.compact(fe)
    del fe
    np.testing.assert_array_equal(_np(enc.freq_flags), ff)
    np.testing.assert_array_equal(_np(enc.freq_codes), ED.quantize(vf, enc.step_f))
    enc.spat_edits = enc.freq_edits = None
    torch.cuda.empty_cache()
    say("[edits] decoding and FP64 re-verification")
    y = F.decode(xb, enc)
    d = y.double() - x.double()
    ms = float(d.abs().max())
    Dk = torch.fft.rfftn(d)
    mf = float(torch.maximum(Dk.real.abs().max(), Dk.imag.abs().max()))
    say(f"[edits] decoded: max|y-x| {ms / p.E:.6f} E, max spectral {mf / p.Delta:.6f} Delta")
    assert ms <= p.E and mf <= p.Delta
