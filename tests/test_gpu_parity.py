"""GPU parity of the HIP correction path against the FP64 CPU oracle.

Every call goes through the C ABI (``paper_2601_01596_amd.ffcz`` -> libffcz.so).
Tolerances (derived from the arithmetic of each precision):
  FP64: rounds and every per-check violation count equal to the oracle's;
        max|y_gpu - y_orc| <= 1e-12 * max|y_orc|.
  FP32: rounds equal or off by one (then the oracle is re-run for the GPU's
        round count with fixed rounds); max|y_gpu - y_orc| <= 1e-5 * max|y_orc|;
        per-check violation counts within 0.1% (+2).
  Both: the FP64 re-verification of the output passes.
"""

import numpy as np
import pytest

from oracle import ffcz as O
from paper_2601_01596_amd import ffcz as F
from paper_2601_01596_amd import workloads as W
from tests.gpu_util import rel_err, run_gpu, unpack_masks

pytestmark = pytest.mark.gpu


def _problem(shape, seed, dtype, q=90.0, r=1e-2, alpha=2.0):
    x = W.grf(shape, alpha, seed) if len(shape) > 1 or shape[0] > 4 else np.random.default_rng(seed).standard_normal(shape)
    return W.make_problem("t", x, dtype, r, q, 200)


def _check_fp64(p, y, res, orc):
    assert res.status == F.OK, (res.status, F.ffcz_last_error())
    assert res.stats["rounds"] == orc.rounds
    assert rel_err(y, orc.y) <= 1e-12
    assert res.stats["max_spatial_err"] <= p.E and res.stats["max_spectral_err"] <= p.Delta


def _check_fp32(p, y, res, orc):
    assert res.status == F.OK, (res.status, F.ffcz_last_error())
    k = res.stats["rounds"]
    if k != orc.rounds:
        assert abs(k - orc.rounds) <= 1
        orc = O.correct(p.x, p.xb, p.E, p.Delta, k, mu=res.stats["margin_used"], fixed=True)
    assert rel_err(y, orc.y) <= 1e-5
    ms, mf, nv, ok = O.verify(p.x, y, p.E, p.Delta)
    assert ok and nv == 0


def test_grf64_fp64_matches_oracle_counts_and_values():
    # 64^3 FP64 GRF, k^-2, E = 1e-3 range, Delta at the 90th percentile, cap 200
    p = W.config_grf_fp64(64)
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter, record_viol=True)
    orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter)
    _check_fp64(p, y, res, orc)
    viol = res.viol.cpu().numpy()[: orc.rounds + 1]
    assert list(viol) == orc.viol
    assert res.stats["s_guard"] == orc.s_clipped[0]
    assert res.stats["s_clipped_total"] == sum(orc.s_clipped[1:])
    assert res.stats["f_viol_initial"] == orc.viol[0]


SHAPES = [(16, 32, 64), (8, 8, 8), (4, 16, 128), (32, 64), (128, 16), (64, 4096), (256,), (4096,), (2, 4, 8),
          (1, 64, 32), (64, 1, 32), (16, 16, 2), (512, 8)]


@pytest.mark.parametrize("shape", SHAPES)
def test_shapes_fp64(shape):
    p = _problem(shape, 7, np.float64)
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter, record_viol=True)
    orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter)
    _check_fp64(p, y, res, orc)
    assert list(res.viol.cpu().numpy()[: orc.rounds + 1]) == orc.viol


@pytest.mark.parametrize("shape", SHAPES)
def test_shapes_fp32(shape):
    p = _problem(shape, 11, np.float32)
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter, record_viol=True)
    orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter, mu=res.stats["margin_used"])
    _check_fp32(p, y, res, orc)
    # the violation count of every check both ran, within 0.1 % (+2)
    v = res.viol.cpu().numpy()
    for k in range(min(res.stats["rounds"], orc.rounds) + 1):
        assert abs(int(v[k]) - orc.viol[k]) <= 2 + 1e-3 * orc.viol[k], (k, int(v[k]), orc.viol[k])


@pytest.mark.parametrize("shape", [(2048, 64), (2048, 4, 8)])
def test_leading_2048_fp32(shape):
    # 2048 is the longest leading extent in FP32 (FP64 stops at 1024); its FP64 check runs
    # the 2048-point column transform in FP64
    test_shapes_fp32(shape)


@pytest.mark.parametrize("dt,shape", [(np.float32, (2048, 2048)), (np.float64, (1024, 4096))])
def test_largest_2d_extents(dt, shape):
    O.set_workers(max(1, min(16, O.default_workers())))
    p = _problem(shape, 13, dt)
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
    mu = res.stats["margin_used"]
    orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter, mu=mu)
    (_check_fp64 if dt == np.float64 else _check_fp32)(p, y, res, orc)


def test_lognormal64_fp32_and_fp64():
    # the 512^3 lognormal recipe (k^-2.5, E = 1e-4 range, 95th percentile) at 64^3
    for dt in (np.float32, np.float64):
        p = W.config_lognormal(64, dt)
        y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
        mu = res.stats["margin_used"]
        orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter, mu=mu)
        (_check_fp64 if dt == np.float64 else _check_fp32)(p, y, res, orc)


def test_max_iter_zero_and_one_not_converged():
    p = _problem((16, 16, 16), 3, np.float64, q=50.0)
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, 0)
    assert res.status == F.NOT_CONVERGED and res.stats["rounds"] == 0
    orc = O.correct(p.x, p.xb, p.E, p.Delta, 0)
    assert rel_err(y, orc.y) <= 1e-12
    y, res = run_gpu(p.x, p.xb, p.E, p.Delta, 1)
    orc = O.correct(p.x, p.xb, p.E, p.Delta, 1)
    assert res.stats["rounds"] == 1 and res.status == orc.status
    assert rel_err(y, orc.y) <= 1e-12


def test_zero_rounds_when_already_inside_both_cubes():
    g = np.random.default_rng(4)
    x = g.standard_normal((8, 16, 32))
    E = 0.01
    xb = x + g.uniform(-0.5 * E, 0.5 * E, x.shape)
    y, res = run_gpu(x, xb, E, x.size * E, 10)
    assert res.status == F.OK and res.stats["rounds"] == 0 and res.stats["f_viol_initial"] == 0
    assert rel_err(y, xb) <= 1e-13


def test_nonfinite_input_is_reported():
    p = _problem((16, 16, 16), 5, np.float32)
    xb = p.xb.copy()
    xb[3, 4, 5] = np.nan
    _, res = run_gpu(p.x, xb, p.E, p.Delta, 20)
    assert res.status == F.E_NONFINITE
    assert res.stats["nonfinite"] == 1


def test_argument_errors():
    import torch
    x = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    xb = torch.zeros_like(x)
    r = F.correct(x, xb, -1.0, 1.0, 5, check=False)
    assert r.status == F.E_INVALID
    r = F.correct(x, xb, 1.0, float("nan"), 5, check=False)
    assert r.status == F.E_INVALID
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    # the binding refuses a short workspace before the call; the C ABI refuses it too
    with pytest.raises(F.FFCzError) as ei:
        F.correct(x, xb, 1.0, 1.0, 5, ws=ws, check=False)
    assert ei.value.status == F.E_WORKSPACE
    y = torch.empty_like(x)
    st = F.ffcz_correct(F.F32, (8, 8, 8), x.data_ptr(), xb.data_ptr(), y.data_ptr(), 1.0, 1.0, 5, None,
                        ws.data_ptr(), ws.numel(), 0, None)
    assert st == F.E_WORKSPACE
    bad = torch.zeros((8, 6, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(F.FFCzError):
        F.correct(bad, bad.clone(), 1.0, 1.0, 5)


def test_deterministic_bitwise():
    p = W.config_lognormal(32, np.float32)
    y1, r1 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
    y2, r2 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
    assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32))
    assert r1.stats == r2.stats


@pytest.mark.parametrize("dt,shape,mode", [(np.float64, (16, 16, 64), 1), (np.float32, (16, 16, 64), 1),
                                           (np.float32, (8, 8, 512), 4), (np.float32, (8, 16, 256), 4)])
def test_fixed_rounds_masks_match_oracle(dt, shape, mode):
    """Clip keep-masks equal the oracle's; in FP32 a bit may differ only where the
    oracle's pre-clip value lies within FP32 noise (1e-5 relative) of its bound.  Mode 4
    runs the direct last-axis passes (rows of 128 and 256 entries)."""
    p = _problem(shape, 21, dt, q=85.0, r=5e-2)
    K = 5
    try:
        F.ffcz_set_tuning(mode)
        y, res = run_gpu(p.x, p.xb, p.E, p.Delta, K, fixed=True, record_masks=True)
    finally:
        F.ffcz_set_tuning(1)
    assert res.stats["rounds"] == K
    mu = res.stats["margin_used"]
    orc = O.correct(p.x, p.xb, p.E, p.Delta, K, mu=mu, fixed=True, record_masks=True)
    assert rel_err(y, orc.y) <= (1e-12 if dt == np.float64 else 1e-5)
    gm = unpack_masks(res.masks.cpu().numpy(), p.x.shape, K)
    _masks_differ_only_at_bounds(p, dt, mu, K, gm, orc.masks)


def _masks_differ_only_at_bounds(p, dt, mu, K, gm, om):
    """The GPU's keep-masks gm equal the oracle's om; in FP32 a bit may differ only where the
    oracle's pre-clip value lies within FP32 noise (1e-5 relative) of its bound (the clip
    decision of Eq. 2's projections at the bound is a rounding question).  Returns the number
    of differing bits."""
    Ep = p.E * (1 - mu)
    Dp = O.spectral_thresholds(p.Delta, mu, dt)[1]
    np.testing.assert_array_equal(gm.s[0], om.s[0])  # guard clip runs in FP64
    nbad = 0
    for k in range(1, K + 1):
        prev = O.correct(p.x, p.xb, p.E, p.Delta, k - 1, mu=mu, fixed=True, verify_output=False).eps
        d = O.fft(prev)                                   # pre-clip spectrum of block k
        pre_s = O.ifft(O.project_f(d, Dp)[0], p.x.shape)  # pre-clip spatial error of block k
        pairs = ((gm.s[k], om.s[k], pre_s, Ep), (gm.f_re[k], om.f_re[k], d.real, Dp),
                 (gm.f_im[k], om.f_im[k], d.imag, Dp))
        for a, b, pre, thr in pairs:
            bad = a != b
            nbad += int(bad.sum())
            if dt == np.float64:
                assert not bad.any(), (k, int(bad.sum()))
            else:
                gap = np.abs(np.abs(pre[bad]) - thr)
                assert np.all(gap <= 1e-5 * thr), (k, int(bad.sum()), float(gap.max(initial=0)) / thr)
    return nbad


@pytest.mark.parametrize("dt,shape", [(np.float64, (16, 16, 64)), (np.float32, (16, 16, 64)),
                                      (np.float64, (32, 128)), (np.float32, (8, 32, 32))])
def test_backward_matches_oracle_adjoint(dt, shape, mode=1):
    import torch
    p = _problem(shape, 31, dt, q=85.0, r=5e-2)
    K = 4
    try:
        F.ffcz_set_tuning(mode)
        y, res = run_gpu(p.x, p.xb, p.E, p.Delta, K, fixed=True, record_masks=True)
        g = np.random.default_rng(32).standard_normal(shape).astype(dt)
        gb = F.correct_backward(torch.from_numpy(g).cuda(), res.masks, K).cpu().numpy()
    finally:
        F.ffcz_set_tuning(1)
    gm = unpack_masks(res.masks.cpu().numpy(), shape, K)
    ref = O.adjoint(gm, g.astype(np.float64))          # oracle fed the GPU's own masks
    tol = 1e-12 if dt == np.float64 else 1e-5
    assert rel_err(gb, ref) <= tol
    mu = res.stats["margin_used"]
    orc = O.correct(p.x, p.xb, p.E, p.Delta, K, mu=mu, fixed=True, record_masks=True)
    # the oracle's own trajectory: its masks equal the GPU's but for FP32 clip decisions at a
    # bound, and where they all agree its adjoint is the GPU's
    nbad = _masks_differ_only_at_bounds(p, dt, mu, K, gm, orc.masks)
    if nbad == 0:
        ref2 = O.adjoint(orc.masks, g.astype(np.float64))
        rel_l2 = np.linalg.norm(gb - ref2) / np.linalg.norm(ref2)
        assert rel_l2 <= (1e-12 if dt == np.float64 else 1e-4)


@pytest.mark.parametrize("shape", [(16, 16, 256), (8, 16, 512), (32, 256), (2, 4, 256), (2, 4, 512)])
def test_direct_last_axis_backward_matches_oracle_adjoint(shape):
    # mode 4: the forward and the adjoint run the direct last-axis passes (rows of 128 and
    # 256 entries); the last two shapes have fewer rows than one block (8 of 32 and of 16), so
    # lanes past the last row repeat it, mask bits included
    test_backward_matches_oracle_adjoint(np.float32, shape, mode=4)


def test_backward_dot_product_identity():
    # <J u, v> = <u, J^T v> with the recorded masks: J u from the oracle's JVP, J^T v from the GPU
    import torch
    p = _problem((16, 32, 32), 41, np.float64, q=85.0, r=5e-2)
    K = 3
    _, res = run_gpu(p.x, p.xb, p.E, p.Delta, K, fixed=True, record_masks=True)
    gm = unpack_masks(res.masks.cpu().numpy(), p.x.shape, K)
    g = np.random.default_rng(1)
    u = g.standard_normal(p.x.shape)
    v = g.standard_normal(p.x.shape)
    jtv = F.correct_backward(torch.from_numpy(v).cuda(), res.masks, K).cpu().numpy()
    lhs = np.sum(O.forward_fixed_masks(gm, u) * v)
    rhs = np.sum(u * jtv)
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1.0)


def test_autograd_function_gradient():
    import torch
    p = _problem((8, 16, 32), 51, np.float32, q=85.0, r=5e-2)
    x = torch.from_numpy(p.x).cuda()
    xb = torch.from_numpy(p.xb).cuda().requires_grad_(True)
    w = torch.from_numpy(np.random.default_rng(52).standard_normal(p.x.shape).astype(np.float32)).cuda()
    y = F.FFCzCorrect.apply(xb, x, p.E, p.Delta, 3)
    (y * w).sum().backward()
    r = F.correct(x, xb.detach(), p.E, p.Delta, 3, fixed=True, verify=False, record_masks=True)
    ref = F.correct_backward(w, r.masks, 3)
    assert torch.equal(xb.grad, ref)


@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 128)])
def test_graph_replays_match_plain_launches(shape):
    """The round chunk captured in a hipGraph and replayed gives the plain-launch result,
    bit for bit, on every replay, with unrelated device work and synchronisations between."""
    import torch
    p = _problem(shape, 61, np.float32, q=90.0)
    x = torch.from_numpy(p.x).cuda()
    xb = torch.from_numpy(p.xb).cuda()
    ref = F.correct(x, xb, p.E, p.Delta, p.max_iter, graph=False, chunk=2)
    for rep in range(4):
        junk = torch.randn(1 << 20, device="cuda").sum()  # other work between replays
        torch.cuda.synchronize()
        r = F.correct(x, xb, p.E, p.Delta, p.max_iter, graph=True, chunk=2)
        torch.cuda.synchronize()
        assert r.status == ref.status and r.stats == ref.stats, rep
        assert torch.equal(r.y, ref.y), rep
        del junk


@pytest.mark.parametrize("nbytes", [16, 1000, (1 << 20) + 48, (64 << 20) + 7])
def test_copy_kernel_bit_exact(nbytes):
    import torch
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=torch.Generator().manual_seed(nbytes)).cuda()
    dst = torch.zeros_like(src)
    F.copy_(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


@pytest.mark.parametrize("pattern", ["x", "y"])
def test_strided_copy_bit_exact(pattern):
    # rows of 2064 bytes (the last 128-byte tile holds 16 of them) at a pitch of 2176 bytes,
    # 9 rows per plane, 37 planes padded by 128 bytes: the x-pass pattern walks the planes,
    # the y-pass pattern the rows; every other byte stays untouched
    import torch
    nrow, pitch, nplane, row_bytes = 9, 2176, 37, 2064
    plane = nrow * pitch + 128
    args = (nplane, plane, nrow, pitch) if pattern == "x" else (nrow, pitch, nplane, plane)
    size = nplane * plane
    src = torch.randint(0, 256, (size,), dtype=torch.uint8, generator=torch.Generator().manual_seed(91))
    exp = np.zeros(size, dtype=np.uint8)
    s_np = src.numpy()
    for pl in range(nplane):
        for r in range(nrow):
            o = pl * plane + r * pitch
            exp[o:o + row_bytes] = s_np[o:o + row_bytes]
    dst = torch.zeros(size, dtype=torch.uint8).cuda()
    F.copy_columns_(dst, src.cuda(), *args, row_bytes)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), exp)


@pytest.mark.parametrize("dt,shape", [(np.float32, (32, 64, 128)), (np.float64, (64, 32, 256)),
                                      (np.float32, (256, 512)), (np.float32, (2048, 128)),
                                      (np.float32, (2, 4, 512)), (np.float32, (4, 8, 1024)),
                                      (np.float32, (64, 2048)), (np.float32, (8, 4096)),
                                      (np.float32, (256, 256, 512))])
def test_tile_variants_bit_identical(dt, shape):
    # every tiling the tuner may pick computes the same bits: default tiles vs the narrowest
    # (mode 2), masks included
    p = _problem(shape, 71, dt)
    K = 3
    runs = []
    try:
        for mode in (0, 2):
            F.ffcz_set_tuning(mode)
            y, r = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter, record_viol=True)
            yk, rk = run_gpu(p.x, p.xb, p.E, p.Delta, K, fixed=True, record_masks=True)
            runs.append((y, r, rk.masks.cpu().numpy()))
    finally:
        F.ffcz_set_tuning(1)
    y0, r0, m0 = runs[0]
    for y1, r1, m1 in runs[1:]:
        assert r0.status == F.OK and r1.status == F.OK
        assert np.array_equal(y0.view(np.uint8), y1.view(np.uint8))
        assert r0.stats == r1.stats
        assert np.array_equal(r0.viol.cpu().numpy(), r1.viol.cpu().numpy())
        assert np.array_equal(m0, m1)


@pytest.mark.parametrize("dt,shape", [(np.float32, (32, 64, 512)), (np.float64, (16, 32, 256)),
                                      (np.float32, (8, 4, 256)), (np.float32, (2, 512)),
                                      (np.float32, (1024,)), (np.float64, (4, 16)),
                                      (np.float32, (16, 2048)), (np.float64, (4, 4096))])
def test_output_independent_of_verification(dt, shape):
    # rows of up to 512 entries close in one pass that also starts the FP64 verification
    # (longer rows keep two passes); y is the same bits with verification off, and the
    # verified maxima match the oracle's FP64 re-verification of that y
    p = _problem(shape, 83, dt)
    y1, r1 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
    y0, r0 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter, verify=False)
    assert r1.status == F.OK and r0.status in (F.OK, F.NOT_CONVERGED)
    assert np.array_equal(y1.view(np.uint8), y0.view(np.uint8))
    assert r1.stats["rounds"] == r0.stats["rounds"]
    ms, mf, _, _ = O.verify(p.x, y1, p.E, p.Delta)
    assert r1.stats["max_spatial_err"] == pytest.approx(ms, rel=1e-12, abs=0.0)
    assert r1.stats["max_spectral_err"] == pytest.approx(mf, rel=1e-9)


@pytest.mark.parametrize("mode,dt,shape", [(3, np.float32, (32, 64, 256)), (3, np.float64, (16, 32, 512)),
                                           (3, np.float32, (128, 1024)), (3, np.float64, (64, 128)),
                                           (3, np.float32, (1024, 64)), (3, np.float32, (2048, 32)),
                                           (3, np.float32, (8, 1024, 16)), (3, np.float64, (1024, 32)),
                                           (4, np.float32, (16, 32, 512)), (4, np.float32, (2, 4, 512)),
                                           (4, np.float32, (256, 512)), (4, np.float64, (16, 32, 512)),
                                           (4, np.float32, (16, 32, 256)), (4, np.float32, (4, 8, 256)),
                                           (4, np.float32, (64, 256))])
def test_rounding_plans_match_oracle(mode, dt, shape):
    # the radix-8 last-axis plan (mode 3; long columns included) and the direct last-axis loop
    # pass (mode 4, FP32 rows of 256 entries; FP64 runs the narrow tiles) round differently
    # from the default plan but meet the same bars
    p = _problem(shape, 77, dt)
    try:
        F.ffcz_set_tuning(mode)
        y, res = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter, record_viol=True)
    finally:
        F.ffcz_set_tuning(1)
    orc = O.correct(p.x, p.xb, p.E, p.Delta, p.max_iter, mu=res.stats["margin_used"])
    (_check_fp64 if dt == np.float64 else _check_fp32)(p, y, res, orc)
    if dt == np.float64:
        assert list(res.viol.cpu().numpy()[: orc.rounds + 1]) == orc.viol


def test_tuning_cache_file_roundtrip(tmp_path):
    import json
    path = tmp_path / "plans.json"
    p = _problem((64, 64, 128), 73, np.float32)
    try:
        F.ffcz_clear_tuning()
        assert F.ffcz_set_tuning(1, str(path)) == F.OK
        y0, r0 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
        doc = json.loads(path.read_text())
        keys = list(doc["entries"])
        nvar = {"y": 2, "x": 2, "z": 4}
        assert len(keys) == 3 and all(len(doc["entries"][k]["ms"]) == nvar[k.split()[2]] for k in keys), doc
        assert {k.split()[2] for k in keys} == {"y", "x", "z"}
        # a fresh table read back from the file takes the same decisions without timing
        F.ffcz_clear_tuning()
        assert F.ffcz_set_tuning(1, str(path)) == F.OK
        y1, r1 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
        assert np.array_equal(y0.view(np.uint8), y1.view(np.uint8))
        assert F.ffcz_set_tuning(5) == F.E_INVALID
    finally:
        F.ffcz_set_tuning(1, "")
        F.ffcz_clear_tuning()


@pytest.mark.parametrize("shape, offset", [((8,), 0), ((4096,), 1), ((16, 4096), 3), ((32, 64), 2),
                                           ((64, 64, 64), 0), ((2, 4, 128), 1), ((1024, 2048), 0)])
def test_device_margin_matches_oracle(shape, offset):
    """The FP32 margin derived on the device (slot partial sums of ulp(x)^2, folded in a fixed
    order) against the oracle's formula, from unaligned starts too.  A correction that derives
    its own margin reports exactly the suggested value."""
    import torch
    rng = np.random.default_rng(sum(shape) + offset)
    n = int(np.prod(shape))
    x = (rng.standard_normal(n + offset) * 10.0 ** rng.uniform(-3, 3, n + offset)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()[offset:].reshape(shape)
    D = 0.37
    ws = F.workspace(F.F32, shape, 4, xt.device)
    stream = torch.cuda.current_stream().cuda_stream
    mu = F.ffcz_suggest_margin(F.F32, shape, xt.data_ptr(), D, ws.data_ptr(), ws.numel(), stream)
    ref = O.suggest_margin(x[offset:].reshape(shape), D)
    assert abs(mu - ref) <= 1e-12 * ref, (mu, ref)
    if offset == 0:
        xb = (xt + 1e-3).contiguous()
        r = F.correct(xt, xb, 2e-3, D, 4, ws=ws)
        assert r.stats["margin_used"] == mu
    mu64 = F.ffcz_suggest_margin(F.F64, shape, xt.data_ptr(), D, ws.data_ptr(), ws.numel(), stream)
    assert mu64 == 2.0 ** -16


def test_device_margin_ragged_lengths_in_a_batch():
    """Batched 1D members of any length: slices of a multiple of 4 points with a ragged last
    slot; each member's margin against the oracle's formula."""
    import torch
    rng = np.random.default_rng(77)
    lens = [2, 3, 7, 4097, 16385, 100003, 262147]
    mem, xs = [], []
    for n in lens:
        x = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)).astype(np.float32)
        xs.append(x)
        xt = torch.from_numpy(x).cuda()
        mem.append((xt, (xt + 1e-3).contiguous(), 2e-3, 0.37 * np.sqrt(n)))
    _, st, stats = F.correct_batched(mem, 4, check=False)
    for x, m, s in zip(xs, mem, stats):
        ref = O.suggest_margin(x, m[3])
        assert abs(s["margin_used"] - ref) <= 1e-12 * ref, (x.size, s["margin_used"], ref)


def test_library_loaded_before_torch():
    """A process that loads the library before it imports torch (the binding loads torch's
    HIP runtime first, so there is one runtime in the process): one small correction in a
    fresh interpreter, checked for status OK."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2601_01596_amd import ffcz as F\n"
            "F.ffcz_set_tuning(1)\n"
            "import torch\n"
            "g = torch.Generator(device='cpu').manual_seed(5)\n"
            "x = torch.randn(8, 16, 32, dtype=torch.float64, generator=g).cuda()\n"
            "xb = (x + 1e-3 * torch.randn(8, 16, 32, dtype=torch.float64, generator=g).cuda()).contiguous()\n"
            "r = F.correct(x, xb, 2e-3, 0.05, 20, check=False)\n"
            "print('status', r.status, F.ffcz_last_error(), flush=True)\n")
    env = dict(os.environ, PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                         timeout=180)
    lines = [ln for ln in out.stdout.splitlines() if ln.startswith("status")]
    assert out.returncode == 0 and lines, (out.returncode, out.stdout[-2000:], out.stderr[-2000:])
    assert lines[-1].split()[1] in (str(F.OK), str(F.NOT_CONVERGED)), lines[-1]


def test_profile_select_times_only_the_chosen_passes():
    # per-launch events around the selected pass kind only; the same launches of that kind
    # are counted as with every kind timed, and the output does not change
    p = _problem((32, 32, 64), 91, np.float32)
    try:
        F.ffcz_profile_select(["x_pass"])
        F.ffcz_profile_enable(True)
        y1, r1 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
        sel = F.ffcz_profile_read()
        F.ffcz_profile_select(None)
        y2, r2 = run_gpu(p.x, p.xb, p.E, p.Delta, p.max_iter)
        full = F.ffcz_profile_read()
    finally:
        F.ffcz_profile_enable(False)
        F.ffcz_profile_select(None)
    assert r1.status == F.OK and r2.status == F.OK
    assert np.array_equal(y1.view(np.uint8), y2.view(np.uint8))
    assert sel["x_pass"][1] == full["x_pass"][1] == r1.stats["rounds"] + 1
    assert sel["x_pass"][0] > 0.0
    assert all(v[1] == 0 for k, v in sel.items() if k != "x_pass")
    assert full["init"][1] == 1 and full["finalize"][1] == 1 and full["verify_x"][1] == 1
