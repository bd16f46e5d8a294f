"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a
brute-force DFT (Eq. 1), Parseval, Hermitian symmetry (Sec. IV-A), the
projection identities of a Euclidean projection, Fejer monotonicity of POCS
(Sec. III), the two regime closed forms (Sec. V, Table 3 discussion; Eq. 4),
hand-worked cases of Alg. 1, a dense O(N^2) re-implementation of the loop,
and finite differences of the forward map for the adjoint.
"""

import math
import os

import numpy as np
import pytest

from oracle import dense, ffcz, spectrum
from paper_2601_01596_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SHAPES_TINY = [(1,), (2,), (3,), (5,), (8,), (4, 6), (5, 6, 7), (8, 8, 8), (3, 4, 5), (2, 1, 3)]


def rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("shape", SHAPES_TINY)
def test_fft_matches_bruteforce_dft(shape):
    e = rng(1).standard_normal(shape)
    full = dense.dense_fft(e)
    half = ffcz.fft(e)
    np.testing.assert_allclose(half, full[..., : shape[-1] // 2 + 1], rtol=0, atol=1e-12)
    back = ffcz.ifft(half, shape)
    np.testing.assert_allclose(back, e, rtol=0, atol=1e-13)


def test_dft_sign_and_scale_on_a_single_tone():
    # Eq. 1: x_n = exp(+2 pi i m n / N) has X_k = N at k = m and 0 elsewhere; for the
    # real cosine the half-spectrum holds N/2 at k = m.
    N, m = 16, 3
    n = np.arange(N)
    X = ffcz.fft(np.cos(2 * np.pi * m * n / N))
    expect = np.zeros(N // 2 + 1, complex)
    expect[m] = N / 2
    np.testing.assert_allclose(X, expect, atol=1e-12)
    X = ffcz.fft(np.sin(2 * np.pi * m * n / N))
    expect[m] = -1j * N / 2   # negative exponent sign of Eq. 1
    np.testing.assert_allclose(X, expect, atol=1e-12)


@pytest.mark.parametrize("shape", [(7,), (8,), (6, 5), (4, 6, 8), (5, 3, 7)])
def test_parseval(shape):
    e = rng(2).standard_normal(shape)
    D = ffcz.fft(e)
    n = shape[-1]
    w = np.full(D.shape[-1], 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    lhs = float(np.sum(w * np.abs(D) ** 2))
    rhs = e.size * float(np.sum(e * e))
    assert abs(lhs - rhs) <= 1e-12 * rhs


@pytest.mark.parametrize("shape", [(8,), (7,), (4, 6), (5, 4, 6), (3, 5, 5)])
def test_half_spectrum_clip_equals_full_spectrum_clip(shape):
    # Hermitian symmetry (Sec. IV-A): clipping the stored half equals clipping all N
    # coefficients; the full clip stays Hermitian so its inverse is real.
    e = rng(3).standard_normal(shape)
    Dp = 0.7
    full = np.fft.fftn(e)
    fc = np.clip(full.real, -Dp, Dp) + 1j * np.clip(full.imag, -Dp, Dp)
    back_full = np.fft.ifftn(fc)
    assert np.max(np.abs(back_full.imag)) < 1e-15
    hc, _, _ = ffcz.project_f(ffcz.fft(e), Dp)
    np.testing.assert_allclose(ffcz.ifft(hc, shape), back_full.real, atol=1e-14)


# ---------------------------------------------------------------- projections

def _pf(eps, Dp):
    return ffcz.ifft(ffcz.project_f(ffcz.fft(eps), Dp)[0], eps.shape)


def _ps(eps, Ep):
    return ffcz.project_s(eps, Ep)[0]


@pytest.mark.parametrize("which", ["f", "s"])
def test_projections_are_euclidean(which):
    r = rng(4)
    shape = (6, 5, 4)
    b = 0.8
    P = (lambda v: _pf(v, b)) if which == "f" else (lambda v: _ps(v, b))
    for _ in range(5):
        v = 2.0 * r.standard_normal(shape)
        pv = P(v)
        # idempotence
        np.testing.assert_allclose(P(pv), pv, atol=1e-13)
        # variational inequality <v - Pv, z - Pv> <= 0 for z in the set
        z = P(3.0 * r.standard_normal(shape))
        assert np.sum((v - pv) * (z - pv)) <= 1e-10
        # non-expansive
        u = 2.0 * r.standard_normal(shape)
        assert np.linalg.norm(P(u) - pv) <= np.linalg.norm(u - v) + 1e-12
    # the f-projection lands in the f-cube
    if which == "f":
        D = ffcz.fft(_pf(5.0 * r.standard_normal(shape), b))
        assert max(np.abs(D.real).max(), np.abs(D.imag).max()) <= b * (1 + 1e-12)


# ---------------------------------------------------------------- the loop

def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    E, D, mu, rounds, v0, v1, sg, y = rows[0]
    return float(E), float(D), float(mu), int(rounds), int(v0), int(v1), int(sg), float(y)


@pytest.mark.parametrize("name,n", [("hand_n4.txt", 4), ("hand_n1.txt", 1)])
def test_hand_worked_cases(name, n):
    E, D, mu, rounds, v0, v1, sg, y = _golden(name)
    x = np.zeros(n)
    xb = np.full(n, E if n == 4 else 3.0)
    r = ffcz.correct(x, xb, E, D, 10, mu=mu)
    assert r.status == ffcz.OK
    assert r.rounds == rounds
    assert r.viol == [v0, v1]
    assert r.s_clipped[0] == sg
    np.testing.assert_array_equal(r.y, np.full(n, y))


def _random_problem(shape, seed, q=80.0, r_=0.05):
    g = rng(seed)
    x = g.standard_normal(shape)
    E = r_ * (x.max() - x.min())
    xb = W.quantize(x, E)
    return x, xb, E, W.spectral_bound(x, xb, q)


@pytest.mark.parametrize("shape,seed", [((8,), 1), ((6, 5), 2), ((4, 4, 4), 3), ((3, 5, 7), 4),
                                        ((2, 3, 4), 5), ((16,), 6), ((8, 8), 7)])
def test_fft_loop_matches_dense_loop(shape, seed):
    x, xb, E, D = _random_problem(shape, seed)
    r = ffcz.correct(x, xb, E, D, 300)
    eps, k, vh, vf, max_imag = dense.dense_correct(x, xb, E, D, 300)
    assert r.rounds == k
    assert r.viol == vh
    assert all((a == 0) == (b == 0) for a, b in zip(vh, vf))
    assert max_imag < 1e-12 * max(1.0, E)
    np.testing.assert_allclose(r.eps, eps, rtol=0, atol=1e-13 * max(E, 1e-300) + 1e-15)


def test_regime_f_cube_inside_s_cube_gives_one_round_closed_form():
    # If sqrt(2) Delta_p <= E_p, every |eps_n| <= sqrt(2) Delta_p after the f-clip, so the
    # s-clip is inactive: one round, no spatial edits (the small-delta rows of Table 3).
    g = rng(7)
    shape = (6, 8, 10)
    E = 1.0
    eps0 = g.uniform(-E, E, shape) * 0.99
    x = g.standard_normal(shape)
    xb = x + eps0
    D = 0.5 * E
    r = ffcz.correct(x, xb, E, D, 50)
    assert r.rounds == 1 and r.status == ffcz.OK
    assert r.s_clipped[1] == 0
    Dp = D * (1 - ffcz.DEFAULT_MU)
    closed = x + ffcz.ifft(ffcz.project_f(ffcz.fft(xb - x), Dp)[0], shape)
    np.testing.assert_allclose(r.y, closed, atol=1e-13)


def test_regime_s_cube_inside_f_cube_gives_zero_rounds():
    # |Re delta|, |Im delta| <= sum |eps_n| <= N E (Eq. 4): with Delta >= N E nothing violates.
    g = rng(8)
    shape = (4, 5, 6)
    E = 0.1
    x = g.standard_normal(shape)
    xb = x + g.uniform(-0.9 * E, 0.9 * E, shape)
    r = ffcz.correct(x, xb, E, x.size * E, 50)
    assert r.rounds == 0 and r.viol == [0] and r.status == ffcz.OK
    np.testing.assert_array_equal(r.y, x + (xb - x))


def test_fejer_monotone_and_both_bounds():
    # 0 lies in both cubes, so by POCS (Sec. III) ||eps|| never grows along the trajectory.
    x, xb, E, D = _random_problem((8, 8, 8), 9, q=90.0)
    norms = []
    for k in range(0, 6):
        r = ffcz.correct(x, xb, E, D, k, fixed=True, verify_output=False)
        norms.append(np.linalg.norm(r.eps))
    assert all(b <= a * (1 + 1e-14) for a, b in zip(norms, norms[1:]))
    r = ffcz.correct(x, xb, E, D, 500)
    assert r.status == ffcz.OK and r.converged
    assert r.max_spatial_err <= E and r.max_spectral_err <= D


def test_resume_from_output_continues_the_trajectory():
    x, xb, E, D = _random_problem((8, 6, 5), 10, q=95.0)
    full = ffcz.correct(x, xb, E, D, 5, fixed=True, verify_output=False)
    a = ffcz.correct(x, xb, E, D, 2, fixed=True, verify_output=False)
    b = ffcz.correct(x, a.y, E, D, 3, fixed=True, verify_output=False)
    np.testing.assert_allclose(b.eps, full.eps, atol=1e-12 * E)


def test_failure_paths():
    x = np.zeros((4, 4))
    xb = np.ones((4, 4)) * 0.5
    r = ffcz.correct(x, xb, 1.0, 0.1, 0)
    assert r.status == ffcz.NOT_CONVERGED and r.rounds == 0
    r = ffcz.correct(x, xb, 1.0, 0.1, 1)
    assert r.rounds == 1
    bad = xb.copy()
    bad[1, 2] = np.nan
    with pytest.raises(ffcz.OracleError) as ei:
        ffcz.correct(x, bad, 1.0, 0.1, 5)
    assert ei.value.status == ffcz.E_NONFINITE
    with pytest.raises(ffcz.OracleError) as ei:
        ffcz.correct(x, xb, -1.0, 0.1, 5)
    assert ei.value.status == ffcz.E_INVALID
    with pytest.raises(ffcz.OracleError) as ei:
        ffcz.correct(x, xb[:3], 1.0, 0.1, 5)
    assert ei.value.status == ffcz.E_SHAPE
    with pytest.raises(ffcz.OracleError) as ei:
        ffcz.correct(np.zeros((2, 2, 2, 2)), np.zeros((2, 2, 2, 2)), 1.0, 0.1, 5)
    assert ei.value.status == ffcz.E_SHAPE


# ---------------------------------------------------------------- FP32 output

def test_closing_clamp_is_minimal():
    g = rng(11)
    x = g.standard_normal(1000).astype(np.float32)
    E = 1e-6
    y = (x.astype(np.float64) + g.uniform(-1.05 * E, 1.05 * E, 1000)).astype(np.float32)
    c = ffcz.closing_clamp(y, x, E)
    d = np.abs(c.astype(np.float64) - x.astype(np.float64))
    assert np.all(d <= E)
    moved = c != y
    # one ulp further away from x would violate again
    back = np.nextafter(c[moved], np.where(c[moved] > x[moved], np.inf, -np.inf).astype(np.float32))
    assert np.all(np.abs(back.astype(np.float64) - x[moved].astype(np.float64)) > E)
    np.testing.assert_array_equal(c[~moved], y[~moved])


def test_fp32_output_meets_both_bounds_in_fp64():
    p = W.config_grf_fp64(24)
    x = p.x.astype(np.float32)
    xb = p.xb.astype(np.float32)
    r = ffcz.correct(x, xb, p.E, p.Delta, 200)
    assert r.y.dtype == np.float32 and r.status == ffcz.OK
    assert r.margin >= ffcz.DEFAULT_MU
    ms, mf, nv, ok = ffcz.verify(x, r.y, p.E, p.Delta)
    assert ok and nv == 0


def test_spectral_thresholds_per_output_precision():
    mu = 3e-5
    assert ffcz.spectral_thresholds(2.0, mu, np.float64) == (2.0, 2.0 * (1.0 - mu))
    dc, dp = ffcz.spectral_thresholds(2.0, mu, np.float32)
    assert dc == pytest.approx(2.0 * (1.0 - mu), rel=1e-15) and dp == pytest.approx(2.0 * (1.0 - 2.0 * mu), rel=1e-15)


def test_fp32_outputs_keep_delta_after_rounding():
    # EEG-like signals whose accepted coefficients sit just below Delta: checking the FP32
    # iterate against Delta itself lets the output rounding lift some of them above it
    for i in (2, 19, 97, 101):
        p = W.config_eeg(i)
        r = ffcz.correct(p.x, p.xb, p.E, p.Delta, 200)
        ms, mf, nv, ok = ffcz.verify(p.x, r.y, p.E, p.Delta)
        assert r.status == ffcz.OK and ok and nv == 0, (i, mf / p.Delta - 1.0)


def test_suggest_margin_formula_on_constant_field():
    # all points share one ulp u: sigma = u / sqrt(12)
    x = np.full((16, 16), 3.0, np.float32)
    u = float(np.spacing(np.float32(3.0)))
    D = 1e-3
    mu = ffcz.suggest_margin(x, D)
    expect = max(2.0 ** -16, 8.0 * (u / math.sqrt(12.0)) * math.sqrt(256 / 2.0) / D)
    assert mu == pytest.approx(expect, rel=1e-12)


def _rounding_noise(x32, eps):
    """Re/Im of DFT(fl32(y) - y) for y = x + eps formed in FP64: the spectral
    perturbation an FP32 output adds (Eq. 3 applied to the rounding errors)."""
    y = x32.astype(np.float64) + eps
    r = y.astype(np.float32).astype(np.float64) - y
    D = ffcz.fft(r)
    # interior last-axis frequencies: no self-conjugate entries, every Re and Im is a
    # sum of N rounding errors weighted by cos^2 or sin^2 averaging 1/2
    inner = D[..., 1: x32.shape[-1] // 2]
    return np.concatenate([inner.real.ravel(), inner.imag.ravel()])


@pytest.mark.parametrize("field", ["grf", "lognormal", "eeg"])
def test_suggest_margin_matches_measured_fp32_rounding_noise(field):
    # The margin is 8 standard deviations of the spectral perturbation that rounding
    # y = x + eps to FP32 causes.  That standard deviation is a property of the data, not
    # of the formula: measure it from DFT(fl32(y) - y) and require suggest_margin's
    # sigma sqrt(N/2) to agree within 5 % both ways (a dropped 1/12 or sqrt(N) for
    # sqrt(N/2) is off by 3.5x or 1.41x).  The largest perturbation must also stay
    # inside the margin, which is what the margin is for.
    if field == "grf":
        x = W.grf((32, 32, 32), 2.0, 21)
    elif field == "lognormal":
        x = W.lognormal((32, 32, 32), 2.5, 22)
    else:
        x = W.eeg_signal(23, 31000)
    x32 = x.astype(np.float32)
    E = W.spatial_bound(x32, 1e-3)
    eps = rng(24).uniform(-E, E, x.shape)
    noise = _rounding_noise(x32, eps)
    measured = float(np.sqrt(np.mean(noise * noise)))
    D = 1.0
    mu = ffcz.suggest_margin(x32, D)
    assert mu > ffcz.DEFAULT_MU and mu < 0.5  # the formula, not a clamp, decides here
    predicted = mu * D / 8.0
    assert predicted == pytest.approx(measured, rel=0.05), (field, predicted / measured)
    assert float(np.max(np.abs(noise))) <= mu * D


# ---------------------------------------------------------------- adjoint

def _fixed_map(x, E, D, K, mu):
    return lambda xb: ffcz.correct(x, xb, E, D, K, mu=mu, fixed=True, verify_output=False).y


def test_adjoint_matches_finite_difference_jacobian():
    # The fixed-round map is piecewise linear in x_hat; away from clip boundaries a
    # central difference gives its Jacobian exactly (up to rounding).
    shape = (6, 6, 8)
    x, xb, E, D = _random_problem(shape, 12, q=85.0, r_=0.1)
    K = 6
    mu = ffcz.DEFAULT_MU
    base = ffcz.correct(x, xb, E, D, K, mu=mu, fixed=True, record_masks=True, verify_output=False)
    f = _fixed_map(x, E, D, K, mu)
    n = x.size
    h = 1e-7 * E
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        J[:, j] = (f(xb + e.reshape(shape)) - f(xb - e.reshape(shape))).ravel() / (2 * h)
    g = rng(13).standard_normal(shape)
    vjp = ffcz.adjoint(base.masks, g).ravel()
    np.testing.assert_allclose(vjp, J.T @ g.ravel(), atol=1e-6 * np.abs(J.T @ g.ravel()).max())
    v = rng(14).standard_normal(shape)
    jvp = ffcz.forward_fixed_masks(base.masks, v).ravel()
    np.testing.assert_allclose(jvp, J @ v.ravel(), atol=1e-6 * np.abs(J @ v.ravel()).max())


def test_adjoint_dot_product():
    x, xb, E, D = _random_problem((6, 5, 8), 15, q=90.0, r_=0.1)
    base = ffcz.correct(x, xb, E, D, 6, fixed=True, record_masks=True, verify_output=False)
    g = rng(16)
    u = g.standard_normal(x.shape)
    v = g.standard_normal(x.shape)
    lhs = np.sum(ffcz.forward_fixed_masks(base.masks, u) * v)
    rhs = np.sum(u * ffcz.adjoint(base.masks, v))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


# ---------------------------------------------------------------- spectrum loss

def test_power_spectrum_bins_sum_to_parseval_total():
    y = rng(17).standard_normal((8, 8, 8))
    P = spectrum.power_spectrum(y, 64)
    Y = np.fft.fftn(y)
    kk = np.sqrt(sum(g * g for g in np.meshgrid(*[np.fft.fftfreq(8) * 8] * 3, indexing="ij")))
    brute = np.array([np.sum(np.abs(Y[np.rint(kk) == b]) ** 2) for b in range(1, 65)])
    np.testing.assert_allclose(P, brute, rtol=1e-12, atol=1e-9)


def test_spectrum_loss_gradient_finite_difference():
    g = rng(18)
    x = g.standard_normal((6, 6, 8))
    y = x + 0.1 * g.standard_normal(x.shape)
    nb = 6
    grad = spectrum.loss_grad(y, x, nb)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (5, 5, 7), (3, 0, 4)]:
        e = np.zeros_like(y)
        e[idx] = h
        fd = (spectrum.loss(y + e, x, nb) - spectrum.loss(y - e, x, nb)) / (2 * h)
        assert fd == pytest.approx(grad[idx], rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------- workloads

def test_workloads_are_seeded_and_hit_the_violation_fraction():
    a = W.config_grf_fp64(16)
    b = W.config_grf_fp64(16)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.xb, b.xb)
    assert np.max(np.abs(a.xb - a.x)) <= a.E * (1 + 1e-12)
    D = ffcz.fft(a.xb - a.x)
    frac = ffcz.count_violations(D, a.Delta) / D.size
    assert abs(frac - 0.10) <= 2.0 / D.size + 1e-3
    g = W.grf((32, 32, 32), 2.0, 1)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12


def test_eeg_and_diffraction_generators():
    L = W.eeg_length(3)
    assert 2 ** 12 <= L <= 2 ** 18
    s = W.eeg_signal(3, 5000)
    assert s.shape == (5000,) and np.all(np.isfinite(s))
    d = W.diffraction_field(1, 64)
    assert d.shape == (64, 64) and d.min() >= 0 and d.max() <= 2e4
