"""Pins of the edit-coding oracle (Alg. 1 edit bookkeeping, CompactEdits, QuantizeEdits,
decoding; Sec. IV-B, IV-D) against what the paper and the mathematics fix:

- the telescoping identity eps_final = (x_hat - x) + spat_edits + IFFT(freq_edits);
- a dense O(N^2) loop over the FULL spectrum with its own bookkeeping (explicit DFT matrix);
- the f-inside-s regime closed form (one round, frequency edits = clip(D) - D) and the
  s-inside-f regime (no edits);
- the hand-worked N = 4 case of Alg. 1 (tests/golden/hand_n4_edits.txt);
- flags/compaction against a plain loop over the coordinates;
- quantisation: hand values, half-to-even, the step/2 error bound;
- the decoder: without quantisation it reproduces x + eps_final; with it, the error obeys
  the triangle-inequality bound, and the decoded output meets both bounds in FP64.
"""

import os

import numpy as np
import pytest

from oracle import dense, edits as ED, ffcz as O
from paper_2601_01596_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(shape, seed, q=85.0, r=0.05, dt=np.float64):
    g = np.random.default_rng(seed)
    x = g.standard_normal(shape).astype(dt)
    E = r * float(x.max() - x.min())
    xb = W.quantize(x, E).astype(dt)
    return x, xb, E, W.spectral_bound(x, xb, q)


@pytest.mark.parametrize("shape,seed", [((16,), 1), ((6, 10), 2), ((8, 8, 8), 3), ((5, 6, 7), 4), ((32,), 5)])
def test_edits_telescope_to_the_final_error(shape, seed):
    x, xb, E, D = _problem(shape, seed)
    r = O.correct(x, xb, E, D, 200, record_edits=True)
    assert r.rounds >= 1
    rebuilt = (xb - x) + r.spat_edits + O.ifft(r.freq_edits, shape)
    np.testing.assert_allclose(rebuilt, r.eps, rtol=0, atol=1e-12 * E)
    # record_edits changes nothing else
    r0 = O.correct(x, xb, E, D, 200)
    np.testing.assert_array_equal(r0.eps, r.eps)
    assert r0.viol == r.viol


@pytest.mark.parametrize("shape,seed", [((8,), 11), ((6, 5), 12), ((4, 4, 4), 13), ((3, 5, 7), 14), ((16,), 15)])
def test_edits_match_dense_full_spectrum_loop(shape, seed):
    x, xb, E, D = _problem(shape, seed, q=80.0)
    Ep, Dc, Dp = ED.encode_thresholds(E, D, 3e-4, 2e-4)
    r = O.correct(x, xb, E, D, 300, record_edits=True, thresholds=(Ep, Dc, Dp))
    eps, k, spat, freq = dense.dense_correct_edits(x, xb, Ep, Dc, Dp, 300)
    assert r.rounds == k and k >= 1
    np.testing.assert_allclose(r.spat_edits, spat, rtol=0, atol=1e-12 * E)
    # the half-spectrum edits are the full-spectrum edits at the kept entries, and the
    # full-spectrum edits are Hermitian (the clip of a Hermitian spectrum is Hermitian)
    half = dense.half_spectrum_indices(shape)
    np.testing.assert_allclose(r.freq_edits.ravel(), freq.ravel()[half], rtol=0, atol=1e-10 * D)
    neg = tuple((-np.indices(shape)) % np.array(shape).reshape((-1,) + (1,) * len(shape)))
    np.testing.assert_allclose(freq, np.conj(freq[neg]), rtol=0, atol=1e-10 * D)


def test_edits_in_the_f_inside_s_regime_are_the_spectral_clip():
    # sqrt(2) Delta_p <= E_p: one round, the s-clip never acts (Sec. V, small-delta rows of
    # Table 3: no active spatial edits), and the frequency edits are clip(D) - D.
    g = np.random.default_rng(21)
    shape = (6, 8, 10)
    x = g.standard_normal(shape)
    xb = x + 0.99 * g.uniform(-1, 1, shape)
    E, D = 1.0, 0.5
    r = O.correct(x, xb, E, D, 50, record_edits=True)
    assert r.rounds == 1
    assert not np.any(r.spat_edits)
    Dk = O.fft(xb - x)
    Dp = D * (1 - O.DEFAULT_MU)
    expect = (np.clip(Dk.real, -Dp, Dp) - Dk.real) + 1j * (np.clip(Dk.imag, -Dp, Dp) - Dk.imag)
    np.testing.assert_allclose(r.freq_edits, expect, rtol=0, atol=1e-12)


def test_no_edits_when_the_s_cube_sits_inside_the_f_cube():
    g = np.random.default_rng(22)
    shape = (4, 5, 6)
    E = 0.1
    x = g.standard_normal(shape)
    xb = x + g.uniform(-0.9 * E, 0.9 * E, shape)
    r = O.correct(x, xb, E, x.size * E, 50, record_edits=True)
    assert r.rounds == 0
    assert not np.any(r.spat_edits) and not np.any(r.freq_edits)


def _golden_edits():
    with open(os.path.join(GOLDEN, "hand_n4_edits.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    return {r[0]: [float(v) for v in r[1:]] for r in rows}


def test_hand_worked_n4_edits_and_codes():
    g = _golden_edits()
    E, D, mu = g["bounds"]
    x = np.zeros(4)
    xb = np.full(4, E)
    r = O.correct(x, xb, E, D, 10, mu=mu, record_edits=True)
    np.testing.assert_array_equal(r.spat_edits, np.array(g["spat_edits"]))
    fe = np.array(g["freq_edits_re"]) + 1j * np.array(g["freq_edits_im"])
    np.testing.assert_array_equal(r.freq_edits, fe)
    ss, sf = ED.step(E), ED.step(D)
    assert (ss, sf) == tuple(g["steps"])
    fs, vs = ED.compact(ED.spatial_coords(r.spat_edits))
    ff, vf = ED.compact(ED.freq_coords(r.freq_edits))
    assert list(fs) == [int(v) for v in g["spat_flags"]]
    assert list(ff) == [int(v) for v in g["freq_flags"]]
    assert list(ED.quantize(vs, ss)) == [int(v) for v in g["spat_codes"]]
    assert list(ED.quantize(vf, sf)) == [int(v) for v in g["freq_codes"]]


def test_compaction_against_a_plain_loop():
    g = np.random.default_rng(23)
    for n in (1, 7, 8, 9, 64, 1000):
        v = g.standard_normal(n) * (g.random(n) < 0.3)
        flags, cv = ED.compact(v)
        assert flags.size == (n + 7) // 8
        exp_flags = [0] * ((n + 7) // 8)
        exp_vals, pos = [], []
        run = 0
        for i in range(n):
            if v[i] != 0.0:
                exp_flags[i // 8] |= 1 << (i % 8)
                exp_vals.append(v[i])
                pos.append(run)   # exclusive prefix count of the flags before i
                run += 1
        assert list(flags) == exp_flags
        np.testing.assert_array_equal(cv, np.array(exp_vals))
        assert pos == list(range(len(exp_vals)))
        assert int(np.unpackbits(flags).sum()) == cv.size
        np.testing.assert_array_equal(ED.expand(flags, cv, n), v)


def test_quantisation_hand_values_and_error_bound():
    st = ED.step(1.0, 16)
    assert st == 2.0 ** -15
    vals = np.array([0.0, st, -st, 2.5 * st, 3.5 * st, -2.5 * st, 0.49 * st, 1e3 * st])
    assert list(ED.quantize(vals, st)) == [0, 1, -1, 2, 4, -2, 0, 1000]
    g = np.random.default_rng(24)
    v = g.uniform(-3, 3, 10000)
    q = ED.quantize(v, ED.step(2.0, 16))
    assert np.max(np.abs(ED.dequantize(q, ED.step(2.0, 16)) - v)) <= ED.step(2.0, 16) / 2
    with pytest.raises(OverflowError):
        ED.quantize(np.array([2.0 ** 40]), 1.0)


def test_encode_margins_hand_values():
    # FP32, max|x| = 1, E = 0.5: ulp(1.5) = 2^-23, so mu_s = 4 * 2^-16 + 2^-23 / 0.5
    x = np.array([1.0, -0.25, 0.5], np.float32)
    mu_s, mu_f = ED.encode_margins(x, 0.5, 1e6, np.float32)
    assert mu_s == 2.0 ** -14 + 2.0 ** -22
    assert mu_f == 2.0 ** -14   # the FP32 rounding margin is below 4 * 2^-16 for this Delta
    mu_s, mu_f = ED.encode_margins(x.astype(np.float64), 0.5, 1.0, np.float64)
    assert mu_s == 2.0 ** -14 + 2.0 ** -52 / 0.5
    assert mu_f == 2.0 ** -14


@pytest.mark.parametrize("shape,seed", [((16, 12), 31), ((8, 8, 8), 32), ((64,), 33)])
def test_decoder_error_shrinks_with_the_code_length(shape, seed):
    # the decoder's distance to x + eps_final is the dequantisation error alone: it obeys
    # step_s/2 + (2 nnz_f / N) step_f/2 and falls by 2^-8 from m = 16 to m = 24
    x, xb, E, D = _problem(shape, seed)
    errs = []
    for m in (16, 24):
        enc = ED.encode(x, xb, E, D, 200, m=m, mus=ED.encode_margins(x, E, D, np.float64))
        y = ED.decode(xb, enc)
        err = float(np.max(np.abs(y - (x + enc.eps))))
        bound = enc.step_s / 2 + 2.0 * enc.freq_codes.size / x.size * enc.step_f / 2
        assert err <= bound * (1 + 1e-9) + 1e-15 * E
        errs.append(err)
    assert errs[1] <= errs[0] * 2.0 ** -6 + 1e-14 * E


@pytest.mark.parametrize("shape,seed,dt", [((16, 12), 41, np.float64), ((16, 16, 16), 42, np.float64),
                                           ((16, 16, 16), 43, np.float32), ((4096,), 44, np.float32),
                                           ((64, 64), 45, np.float32)])
def test_decoded_output_meets_both_bounds_and_the_quantisation_bound(shape, seed, dt):
    if len(shape) == 1:
        x = W.eeg_signal(seed, shape[0]).astype(dt)
        E = 1e-3 * float(x.max() - x.min())
        xb = W.quantize(x, E).astype(dt)
        D = W.spectral_bound(x, xb, 90.0)
    else:
        x, xb, E, D = _problem(shape, seed, q=90.0, r=1e-2, dt=dt)
    enc = ED.encode(x, xb, E, D, 300)
    assert enc.converged
    y = ED.decode(xb, enc)
    assert y.dtype == np.dtype(dt)
    ms, mf, nv, ok = O.verify(x, y, E, D)
    assert ok, (ms / E, mf / D, nv)
    # |decoded - (x + eps)| <= step_s / 2 + (2 nnz_f / N) step_f / 2 + rounding of the output
    N = x.size
    bound = enc.step_s / 2 + 2.0 * enc.freq_codes.size / N * enc.step_f / 2
    bound += float(np.spacing(np.dtype(dt).type(np.max(np.abs(x)) + E)))
    err = np.max(np.abs(y.astype(np.float64) - (x.astype(np.float64) + enc.eps)))
    assert err <= bound * (1 + 1e-9)
    # flags count the non-zero accumulators; codes are the accumulators over the step
    assert int(np.unpackbits(enc.spat_flags).sum()) == enc.spat_codes.size == np.count_nonzero(enc.spat_edits)
    assert int(np.unpackbits(enc.freq_flags).sum()) == enc.freq_codes.size == np.count_nonzero(enc.freq_edits.real) + np.count_nonzero(enc.freq_edits.imag)


def test_paper_shrink_alone_lets_quantisation_error_leak_across_domains():
    # The 64^3 FP64 GRF workload: with the paper's shrink of 2^-m alone, the spatial
    # quantisation error (up to E 2^-m at points the s-clip left on E_p) plus the
    # spatial image of the frequency quantisation error lifts some decoded points above E;
    # the encoder's 4 * 2^-m shrink leaves room for both.
    p = W.config_grf_fp64(64)
    O.set_workers(max(1, min(8, O.default_workers())))
    res = {}
    for safety in (1.0, 4.0):
        enc = ED.encode(p.x, p.xb, p.E, p.Delta, p.max_iter, safety=safety)
        y = ED.decode(p.xb, enc)
        res[safety] = O.verify(p.x, y, p.E, p.Delta)
    ms1, mf1, nv1, ok1 = res[1.0]
    assert not ok1 and ms1 > p.E and nv1 == 0
    assert ms1 <= p.E * (1 + 2.0 ** -16)   # only just above: the leak is of the order of a step
    assert res[4.0][3]
