"""Pins of the generalised-bounds oracle (pointwise E_n and D_k, the disk variant, relative
power-spectrum bounds; footnote to Eq. 2 in Sec. IV-A, Sec. V-B Observation 4) against what
the paper and the mathematics fix:

- constant arrays reproduce the scalar oracle bit for bit;
- a dense loop over the FULL spectrum (explicit DFT matrix, Hermitian-extended bounds, every
  coefficient checked and clipped) gives the same rounds, counts and error;
- the disk and pointwise-box projections: idempotence, the variational inequality of a
  Euclidean projection, non-expansiveness, the radial closed form;
- the per-shell bound: the adversarial error aligned with X (disk) reaches the relative bound
  exactly, the box corners and random errors inside the box stay below it;
- the s-inside-f regime (zero rounds) and the end-to-end guarantee on a GRF.
"""

import math

import numpy as np
import pytest

from oracle import bounds as B
from oracle import dense
from oracle import ffcz as O
from paper_2601_01596_amd import workloads as W


def _problem(shape, seed, r=0.02, q=85.0, dt=np.float64):
    g = np.random.default_rng(seed)
    x = g.standard_normal(shape).astype(dt)
    E = r * float(x.max() - x.min())
    xb = W.quantize(x, E).astype(dt)
    return x, xb, E, W.spectral_bound(x, xb, q)


def _sym_random(shape, seed, lo=0.5, hi=1.5):
    """A positive half-spectrum array with D_{-k} = D_k (a function of the folded frequency)."""
    g = np.random.default_rng(seed)
    full = g.uniform(lo, hi, shape)
    idx = np.indices(shape)
    neg = tuple((-idx[i]) % shape[i] for i in range(len(shape)))
    full = 0.5 * (full + full[neg])
    return full[..., : shape[-1] // 2 + 1]


@pytest.mark.parametrize("shape,seed", [((8, 8, 8), 1), ((6, 10), 2), ((16,), 3), ((5, 6, 7), 4)])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_constant_arrays_reproduce_the_scalar_oracle(shape, seed, dt):
    x, xb, E, D = _problem(shape, seed, dt=dt)
    mu = O.DEFAULT_MU if dt == np.float64 else 3e-4
    a = O.correct(x, xb, E, D, 200, mu=mu)
    b = B.correct(x, xb, np.full(shape, E), np.full(B.half_shape(shape), D), 200, mu=mu)
    assert a.rounds == b.rounds and a.viol == b.viol and a.s_clipped == b.s_clipped
    np.testing.assert_array_equal(a.eps, b.eps)
    np.testing.assert_array_equal(a.y, b.y)


def _full_bounds(Dh, shape):
    """Full-spectrum bounds from a half-spectrum array by Hermitian symmetry."""
    nl = shape[-1]
    idx = np.indices(shape)
    k_last = idx[-1]
    take = tuple(np.where(k_last <= nl // 2, idx[i], (-idx[i]) % shape[i]) for i in range(len(shape)))
    return Dh[take]


def _dense_loop(x, xb, E, Dre, Dim, disk, mu, max_iter):
    """Alg. 1 with the explicit DFT matrix over the full spectrum and pointwise bounds."""
    shape = x.shape
    Wm = dense.dft_matrix(shape)
    N = x.size
    Ep = (E * (1 - mu)).ravel()
    fre, fim = _full_bounds(Dre, shape).ravel(), _full_bounds(Dim, shape).ravel()
    half = dense.half_spectrum_indices(shape)
    eps = (xb - x).ravel().astype(np.float64)
    eps = np.minimum(np.maximum(eps, -Ep), Ep)
    viol, k = [], 0
    while True:
        S = Wm @ eps
        if disk:
            bad = np.abs(S) > fre
        else:
            bad = (np.abs(S.real) > fre) | (np.abs(S.imag) > fim)
        viol.append(int(np.count_nonzero(bad[half])))
        if viol[-1] == 0 or k == max_iter:
            break
        if disk:
            m = np.abs(S)
            dp = fre * (1 - mu)
            S = np.where(m > dp, S * dp / np.where(m > 0, m, 1.0), S)
        else:
            S = np.clip(S.real, -fre * (1 - mu), fre * (1 - mu)) + 1j * np.clip(S.imag, -fim * (1 - mu), fim * (1 - mu))
        e = (np.conj(Wm).T @ S) / N
        eps = np.minimum(np.maximum(e.real, -Ep), Ep)
        k += 1
    return eps.reshape(shape), k, viol


@pytest.mark.parametrize("shape,seed", [((8,), 11), ((6, 5), 12), ((4, 4, 4), 13), ((3, 5, 6), 14), ((4, 6), 15)])
@pytest.mark.parametrize("disk", [False, True])
def test_pointwise_loop_matches_the_dense_full_spectrum_loop(shape, seed, disk):
    x, xb, E0, D0 = _problem(shape, seed, r=0.05, q=75.0)
    g = np.random.default_rng(seed + 100)
    E = E0 * g.uniform(0.6, 1.4, shape)
    Dre = D0 * _sym_random(shape, seed + 200)
    Dim = D0 * _sym_random(shape, seed + 300)
    mu = 1e-4
    r = B.correct(x, xb, E, Dre, 400, D_im=Dim, disk=disk, mu=mu)
    eps, k, viol = _dense_loop(x, xb, E, Dre, Dre if disk else Dim, disk, mu, 400)
    assert r.rounds == k and r.viol == viol
    np.testing.assert_allclose(r.eps, eps, rtol=0, atol=1e-12 * E0)


def test_projection_identities():
    g = np.random.default_rng(31)
    z = g.standard_normal(500) + 1j * g.standard_normal(500)
    Dp = g.uniform(0.2, 1.5, 500)
    Dq = g.uniform(0.2, 1.5, 500)
    for proj in (lambda v: B.project_f_disk(v, Dp)[0], lambda v: B.project_f_box(v, Dp, Dq)[0]):
        p = proj(z)
        np.testing.assert_allclose(proj(p), p, rtol=0, atol=1e-15)            # idempotent
        w = proj(3 * (g.standard_normal(500) + 1j * g.standard_normal(500)))  # points of the set
        assert np.all(((z - p) * np.conj(w - p)).real <= 1e-12)              # variational inequality
        z2 = z + 0.3 * (g.standard_normal(500) + 1j * g.standard_normal(500))
        assert np.all(np.abs(proj(z2) - p) <= np.abs(z2 - z) + 1e-12)        # non-expansive
    # the disk: inside kept, outside moved radially onto the circle
    p, keep = B.project_f_disk(z, Dp)
    m = np.abs(z)
    np.testing.assert_array_equal(keep, m <= Dp)
    np.testing.assert_allclose(np.abs(p[~keep]), Dp[~keep], rtol=1e-14)
    np.testing.assert_allclose(np.angle(p[~keep]), np.angle(z[~keep]), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(p[keep], z[keep])
    # the spatial clip per point
    e = g.standard_normal(300)
    Ep = g.uniform(0.1, 1.0, 300)
    c, kp, n = B.project_s(e, Ep)
    np.testing.assert_array_equal(c, np.clip(e, -Ep, Ep))
    assert n == int(np.count_nonzero(np.abs(e) > Ep))


@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 24), (64,)])
def test_shell_bounds_are_the_largest_that_keep_the_relative_bound(shape):
    g = np.random.default_rng(41)
    x = W.grf(shape, 2.0, 7) + 0.3
    rho = 1e-3
    X = O.fft(x)
    b, w = B.shells(shape)
    P = B.shell_power(X, b, w)
    # disk: the error aligned with X on every entry reaches rho P(b) exactly
    D = B.power_spectrum_bounds(x, rho, disk=True)
    d = D * X / np.abs(X)
    Pd = B.shell_power(X + d, b, w)
    np.testing.assert_allclose((Pd - P) / P, rho, rtol=1e-9)
    # box: the corners aligned with the signs of Re and Im stay within rho P(b) and reach it
    # where |Re X| = |Im X| is common (the bound uses |delta| <= sqrt 2 D)
    D = B.power_spectrum_bounds(x, rho, disk=False)
    d = D * (np.sign(X.real) + 1j * np.sign(X.imag))
    r = (B.shell_power(X + d, b, w) - P) / P
    assert np.all(r <= rho * (1 + 1e-9))
    assert np.max(r) >= 0.7 * rho
    for _ in range(20):
        d = D * (g.uniform(-1, 1, D.shape) + 1j * g.uniform(-1, 1, D.shape))
        r = np.abs(B.shell_power(X + d, b, w) - P) / P
        assert np.all(r <= rho)
    # the weights make the half-spectrum shell sum the full-spectrum one (Parseval per shell)
    np.testing.assert_allclose(P.sum(), x.size * np.sum(x * x), rtol=1e-12)


def test_zero_rounds_when_every_spectral_bound_covers_the_spatial_box():
    # |delta_k| <= sum_n |eps_n| <= sum_n E_n: with min D_k >= sum E_n no coefficient can violate
    g = np.random.default_rng(51)
    shape = (6, 8, 10)
    x = g.standard_normal(shape)
    E = g.uniform(0.05, 0.1, shape)
    xb = x + 0.99 * E * g.uniform(-1, 1, shape)
    Dh = float(E.sum()) * _sym_random(shape, 52, 1.0, 2.0)
    for disk in (False, True):
        r = B.correct(x, xb, E, Dh, 50, disk=disk)
        assert r.rounds == 0 and r.viol == [0] and r.s_clipped == [0]
        np.testing.assert_array_equal(r.y, xb)


@pytest.mark.parametrize("dt,disk", [(np.float64, False), (np.float64, True), (np.float32, False),
                                     (np.float32, True)])
def test_power_spectrum_bound_end_to_end(dt, disk):
    shape = (32, 32, 32)
    x = W.lognormal(shape, 2.5, 61).astype(dt)
    E = W.spatial_bound(x, 1e-3)
    xb = W.quantize(x, E).astype(dt)
    rho = 1e-3
    D = B.power_spectrum_bounds(x, rho, disk=disk)
    # spatially varying E_n as well: twice as tight on the upper half of the first axis
    En = np.full(shape, E)
    En[shape[0] // 2:] *= 0.5
    xb = np.where(np.abs(xb.astype(np.float64) - x) <= En, xb, x).astype(dt)
    r = B.correct(x, xb, En, D, 300, disk=disk)
    assert r.converged and r.rounds >= 1
    rs, rf, nv, ok = B.verify(x, r.y, En, D, disk=disk)
    assert ok, (rs, rf, nv)
    b, w = B.shells(shape)
    P = B.shell_power(O.fft(x.astype(np.float64)), b, w)
    Py = B.shell_power(O.fft(r.y.astype(np.float64)), b, w)
    assert np.max(np.abs(Py - P) / P) <= rho
    # the base reconstruction alone breaks the power-spectrum bound (the correction did work)
    Pb = B.shell_power(O.fft(xb.astype(np.float64)), b, w)
    assert np.max(np.abs(Pb - P) / P) > rho


def test_fp32_margin_uses_the_smallest_bound():
    x = W.grf((16, 16, 16), 2.0, 71).astype(np.float32)
    assert B.suggest_margin(x, 0.37) == O.suggest_margin(x, 0.37)
    assert B.suggest_margin(x, 1e-3, disk=True) == pytest.approx(
        min(0.5, max(O.DEFAULT_MU, math.sqrt(2.0) * O.suggest_margin(x, 1e-3))), rel=1e-15)
