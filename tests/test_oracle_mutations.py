"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in the oracle (a wrong sign, a dropped
term or factor, a wrong bound, mask, index, round cap or clamp) by patching one
of its functions for the duration of the test, then runs the pins of
``test_oracle`` and requires that at least one of them fails.  A mistake that
no pin catches would be a hole in the oracle's pinning.
"""

import math

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import ffcz
from tests import test_oracle as T


def _pins():
    """The pins as plain calls (each raises AssertionError when it fails)."""
    return [
        ("bruteforce_dft", lambda: [T.test_fft_matches_bruteforce_dft(s) for s in [(5,), (4, 6), (3, 4, 5)]]),
        ("single_tone", T.test_dft_sign_and_scale_on_a_single_tone),
        ("parseval", lambda: [T.test_parseval(s) for s in [(7,), (4, 6, 8)]]),
        ("half_vs_full_clip", lambda: T.test_half_spectrum_clip_equals_full_spectrum_clip((5, 4, 6))),
        ("projection_f", lambda: T.test_projections_are_euclidean("f")),
        ("projection_s", lambda: T.test_projections_are_euclidean("s")),
        ("hand_n4", lambda: T.test_hand_worked_cases("hand_n4.txt", 4)),
        ("hand_n1", lambda: T.test_hand_worked_cases("hand_n1.txt", 1)),
        ("dense_loop", lambda: [T.test_fft_loop_matches_dense_loop(s, k) for s, k in [((6, 5), 2), ((4, 4, 4), 3)]]),
        ("regime_f_in_s", T.test_regime_f_cube_inside_s_cube_gives_one_round_closed_form),
        ("regime_s_in_f", T.test_regime_s_cube_inside_f_cube_gives_zero_rounds),
        ("fejer", T.test_fejer_monotone_and_both_bounds),
        ("failure_paths", T.test_failure_paths),
        ("closing_clamp", T.test_closing_clamp_is_minimal),
        ("margin_noise", lambda: [T.test_suggest_margin_matches_measured_fp32_rounding_noise(f)
                                  for f in ("grf", "eeg")]),
        ("adjoint_fd", T.test_adjoint_matches_finite_difference_jacobian),
        ("adjoint_dot", T.test_adjoint_dot_product),
    ]


def _bad_fft_sign(eps):
    return np.conj(sfft.rfftn(eps))


def _bad_ifft_scale(delta, shape):
    return sfft.irfftn(delta, s=tuple(shape)) * float(np.prod(shape)) ** 0.5


def _bad_count_re_only(delta, Delta):
    return int(np.count_nonzero(np.abs(delta.real) > Delta))


def _bad_project_f_bound(delta, Dp):
    re = np.clip(delta.real, -2 * Dp, 2 * Dp)
    im = np.clip(delta.imag, -2 * Dp, 2 * Dp)
    return re + 1j * im, np.abs(delta.real) <= 2 * Dp, np.abs(delta.imag) <= 2 * Dp


def _bad_project_f_sign(orig):
    def f(delta, Dp):
        out, kre, kim = orig(delta, Dp)
        return np.conj(out), kre, kim
    return f


def _bad_project_s_mask(eps, Ep):
    keep = np.abs(eps) <= Ep
    return np.clip(eps, -Ep, Ep), ~keep, int(eps.size - np.count_nonzero(keep))


def _bad_project_s_noop(eps, Ep):
    keep = np.abs(eps) <= Ep
    return np.array(eps, copy=True), keep, int(eps.size - np.count_nonzero(keep))


def _bad_margin_no_twelfth(x, Delta):
    x = np.asarray(x)
    u = ffcz.ulp32(x)
    sigma = math.sqrt(float(np.mean(u * u)))
    return float(min(0.5, max(ffcz.DEFAULT_MU, 8.0 * sigma * math.sqrt(x.size / 2.0) / Delta)))


def _bad_margin_sqrt_n(x, Delta):
    x = np.asarray(x)
    u = ffcz.ulp32(x)
    sigma = math.sqrt(float(np.mean(u * u)) / 12.0)
    return float(min(0.5, max(ffcz.DEFAULT_MU, 8.0 * sigma * math.sqrt(x.size) / Delta)))


def _bad_clamp_none(y32, x, E):
    return np.array(y32, dtype=np.float32, copy=True)


def _bad_clamp_two_steps(orig):
    def f(y32, x, E):
        y = orig(y32, x, E)
        xs = np.asarray(x, dtype=np.float32)
        moved = y != np.asarray(y32, np.float32)
        y[moved] = np.nextafter(y[moved], xs[moved])  # one step too far toward x
        return y
    return f


def _bad_adjoint_index(masks, grad_y):
    shape = grad_y.shape
    K = len(masks.s) - 1
    g = np.asarray(grad_y, dtype=np.float64) * masks.s[K]
    for k in range(K, 0, -1):
        G = ffcz.apply_f_mask(ffcz.fft(g), masks.f_re[k], masks.f_im[k])
        g = ffcz.ifft(G, shape) * masks.s[k]  # should be the mask of block k - 1
    return g


def _bad_adjoint_swap(masks, grad_y):
    shape = grad_y.shape
    K = len(masks.s) - 1
    g = np.asarray(grad_y, dtype=np.float64) * masks.s[K]
    for k in range(K, 0, -1):
        G = ffcz.apply_f_mask(ffcz.fft(g), masks.f_im[k], masks.f_re[k])  # Re and Im masks swapped
        g = ffcz.ifft(G, shape) * masks.s[k - 1]
    return g


def _bad_thresholds(Delta, mu, out_dtype):
    return Delta, Delta  # check and projection both on the unshrunk bound


def _plain(fn):
    return lambda orig: fn


MUTATIONS = {
    "fft_sign": ("fft", _plain(_bad_fft_sign)),
    "ifft_scale": ("ifft", _plain(_bad_ifft_scale)),
    "count_drops_imag": ("count_violations", _plain(_bad_count_re_only)),
    "project_f_bound": ("project_f", _plain(_bad_project_f_bound)),
    "project_f_sign": ("project_f", _bad_project_f_sign),
    "project_s_mask": ("project_s", _plain(_bad_project_s_mask)),
    "project_s_noop": ("project_s", _plain(_bad_project_s_noop)),
    "margin_no_twelfth": ("suggest_margin", _plain(_bad_margin_no_twelfth)),
    "margin_sqrt_n": ("suggest_margin", _plain(_bad_margin_sqrt_n)),
    "clamp_none": ("closing_clamp", _plain(_bad_clamp_none)),
    "clamp_overshoot": ("closing_clamp", _bad_clamp_two_steps),
    "adjoint_index": ("adjoint", _plain(_bad_adjoint_index)),
    "adjoint_swap": ("adjoint", _plain(_bad_adjoint_swap)),
    "no_shrink": ("spectral_thresholds", _plain(_bad_thresholds)),
}


def _run_pins():
    caught = []
    for name, pin in _pins():
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, ffcz.OracleError, FloatingPointError, ValueError, IndexError):
            caught.append(name)
    return caught


@pytest.mark.parametrize("mutation", sorted(MUTATIONS))
def test_planted_mistake_is_caught(mutation, monkeypatch):
    attr, factory = MUTATIONS[mutation]
    monkeypatch.setattr(ffcz, attr, factory(getattr(ffcz, attr)))
    caught = _run_pins()
    assert caught, f"no pin caught the planted mistake {mutation}"


def test_round_cap_off_by_one_is_caught(monkeypatch):
    orig = ffcz.correct

    def early(x, xb, E, Delta, max_iter, **kw):
        return orig(x, xb, E, Delta, max(0, max_iter - 1), **kw)

    monkeypatch.setattr(ffcz, "correct", early)
    assert _run_pins()


def test_missing_guard_clip_is_caught(monkeypatch):
    # the guard clip is the first project_s call of a correction; make it a no-op
    orig = ffcz.project_s
    calls = {"n": 0}

    def skip_first(eps, Ep):
        calls["n"] += 1
        if calls["n"] == 1:
            keep = np.ones(np.shape(eps), bool)
            return np.array(eps, copy=True), keep, 0
        return orig(eps, Ep)

    orig_correct = ffcz.correct

    def correct(*a, **k):
        calls["n"] = 0
        return orig_correct(*a, **k)

    monkeypatch.setattr(ffcz, "project_s", skip_first)
    monkeypatch.setattr(ffcz, "correct", correct)
    assert _run_pins()
