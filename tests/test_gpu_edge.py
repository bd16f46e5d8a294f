"""Edge cases of the method through ffcz_correct on the GPU.

- the hand-worked cases of Alg. 1 (tests/golden: N = 4 and N = 1), whose every
  intermediate value was derived on paper;
- the two regimes with closed forms: f-cube inside the s-cube (one round, no
  spatial clip, y = x + IDFT(clip(DFT(x_hat - x)))) and s-cube inside the f-cube
  (Eq. 4: |Re|, |Im| <= N E, so nothing violates and y = x + (x_hat - x));
- single 1D fields of any length (a 31,000-sample EEG-like record as in Table 1,
  lengths that are not powers of two, a single point), which run on the 1D signal path;
- the x-gradient of the autograd function (dL/dx = dL/dy - dL/dx_hat).
Tolerances as in test_gpu_parity: FP64 1e-12 relative, FP32 1e-5, both bounds in FP64.
"""

import os

import numpy as np
import pytest

from oracle import ffcz as O
from paper_2601_01596_amd import ffcz as F
from paper_2601_01596_amd import workloads as W
from tests.gpu_util import rel_err, run_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    E, D, mu, rounds, v0, v1, sg, y = rows[0]
    return float(E), float(D), float(mu), int(rounds), int(v0), int(v1), int(sg), float(y)


@pytest.mark.parametrize("name,n", [("hand_n4.txt", 4), ("hand_n1.txt", 1)])
def test_hand_worked_cases(name, n):
    # FP64 fields (the worked values use the FP64 thresholds: check Delta, clip Delta (1 - mu))
    dt = np.float64
    E, D, mu, rounds, v0, v1, sg, y = _golden(name)
    x = np.zeros(n, dt)
    xb = np.full(n, E if n == 4 else 3.0, dt)
    yg, res = run_gpu(x, xb, E, D, 10, margin=mu, record_viol=(n == 4))
    assert res.status == F.OK, (res.status, F.ffcz_last_error())
    st = res.stats
    assert st["rounds"] == rounds
    assert st["f_viol_initial"] == v0 and st["f_viol_final"] == v1
    assert st["s_guard"] == sg
    if n == 4:
        assert list(res.viol.cpu().numpy()[: rounds + 1]) == [v0, v1]
    assert np.max(np.abs(yg - y)) <= 1e-12 * abs(y)
    assert st["max_spatial_err"] <= E and st["max_spectral_err"] <= D


def test_regime_f_cube_inside_s_cube_one_round_closed_form():
    # sqrt(2) Delta_p <= E_p: after the f-clip every |eps_n| <= sqrt(2) Delta_p (each of the
    # N coefficients is at most sqrt(2) Delta_p in modulus), so the s-clip never acts
    g = np.random.default_rng(7)
    shape = (8, 8, 16)
    E = 1.0
    x = g.standard_normal(shape)
    xb = x + g.uniform(-E, E, shape) * 0.99
    D = 0.5 * E
    y, res = run_gpu(x, xb, E, D, 50)
    assert res.status == F.OK
    assert res.stats["rounds"] == 1 and res.stats["s_clipped_total"] == 0 and res.stats["s_guard"] == 0
    Dp = D * (1 - O.DEFAULT_MU)
    S = np.fft.rfftn(xb - x)
    closed = x + np.fft.irfftn(np.clip(S.real, -Dp, Dp) + 1j * np.clip(S.imag, -Dp, Dp), s=shape)
    assert rel_err(y, closed) <= 1e-12


def test_regime_s_cube_inside_f_cube_zero_rounds():
    # Eq. 4: |Re delta_k|, |Im delta_k| <= sum_n |eps_n| <= N E; with Delta >= N E nothing violates
    g = np.random.default_rng(8)
    shape = (4, 8, 8)
    E = 0.1
    x = g.standard_normal(shape)
    xb = x + g.uniform(-0.9 * E, 0.9 * E, shape)
    y, res = run_gpu(x, xb, E, x.size * E, 50, record_viol=True)
    assert res.status == F.OK and res.stats["rounds"] == 0
    assert int(res.viol.cpu().numpy()[0]) == 0
    # y = x + eps_0 (the error passes one forward and one inverse transform untouched)
    assert rel_err(y, x + (xb - x)) <= 1e-12


@pytest.mark.parametrize("dt,L", [(np.float32, 31000), (np.float64, 31000), (np.float32, 100003),
                                  (np.float64, 4097), (np.float32, 65536), (np.float64, 3)])
def test_single_1d_field_any_length(dt, L):
    # one EEG-like record through ffcz_correct (the 1D signal path: four-step or Bluestein)
    p = W.make_problem("eeg", W.eeg_signal(60 + L % 97, L), dt, 1e-3, 90.0, 200)
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
    assert res.status == F.OK, (res.status, F.ffcz_last_error())
    st = res.stats
    orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter, mu=st["margin_used"])
    k = st["rounds"]
    if dt == np.float64:
        assert k == orc.rounds and st["f_viol_initial"] == orc.viol[0]
        assert rel_err(y, orc.y) <= 1e-12
    else:
        if k != orc.rounds:
            assert abs(k - orc.rounds) <= 1
            orc = O.correct(p.x, p.xb, p.E, p.Delta, k, mu=st["margin_used"], fixed=True)
        assert rel_err(y, orc.y) <= 1e-5
    ms, mf, nv, ok = O.verify(p.x, y, p.E, p.Delta)
    assert ok and nv == 0
    assert st["max_spatial_err"] == pytest.approx(ms, rel=1e-12)


def test_single_1d_field_refuses_masks():
    import torch
    x = torch.zeros(31000, device="cuda")
    with pytest.raises(F.FFCzError):
        F.correct(x, x + 1e-3, 1e-2, 1.0, 5, record_masks=True)
    r = F.correct(x, x + 1e-3, 1e-2, 1.0, 5, record_viol=True, check=False)
    assert r.status == F.E_INVALID


def test_x_gradient_is_dy_minus_dxhat():
    import torch
    p = W.config_grf_fp64(16)
    x = torch.from_numpy(p.x.astype(np.float32)).cuda().requires_grad_(True)
    xb = torch.from_numpy(p.xb.astype(np.float32)).cuda().requires_grad_(True)
    y = F.FFCzCorrect.apply(xb, x, p.E, p.Delta, 4)
    w = torch.randn_like(y)
    (y * w).sum().backward()
    np.testing.assert_array_equal((w - xb.grad).cpu().numpy(), x.grad.cpu().numpy())
