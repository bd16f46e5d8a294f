"""Batched correction (ffcz_correct_batched) against the oracle, instance by instance.

1D members of any length run one block per signal (four-step FFT; Bluestein for
lengths that are not powers of two); same-shape 2D members share every launch.
Tolerances as in test_gpu_parity: FP64 1e-12 with equal rounds, FP32 1e-5 (rounds
within one), FP64 re-verification of both bounds for every member.
"""


import numpy as np
import pytest

from oracle import ffcz as O
from paper_2601_01596_amd import ffcz as F
from paper_2601_01596_amd import workloads as W
from tests.progress import say
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu




def _member(shape, seed, dt, q=90.0, r=1e-2):
    if len(shape) == 1:
        x = W.eeg_signal(seed, shape[0])
    else:
        x = W.grf(shape, 2.0, seed)
    return W.make_problem("m", x, dt, r, q, 200)


def _run(problems, max_iter=200, **kw):
    import torch
    mem = [(torch.from_numpy(p.x).cuda(), torch.from_numpy(p.xb).cuda(), p.E, p.Delta) for p in problems]
    outs, st, stats = F.correct_batched(mem, max_iter, check=False, **kw)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], st, stats


def _check(p, y, s, dt, max_iter=200):
    """Compare one member with the oracle; returns the oracle's output."""
    assert s["max_spatial_err"] <= p.E and s["max_spectral_err"] <= p.Delta, s
    mu = s["margin_used"]
    orc = O.correct(p.x, p.xb, p.E, p.Delta, max_iter, mu=mu)
    k = s["rounds"]
    if dt == np.float64:
        assert k == orc.rounds, (k, orc.rounds)
        assert rel_err(y, orc.y) <= 1e-12
        assert s["f_viol_initial"] == orc.viol[0]
    else:
        if k != orc.rounds:
            assert abs(k - orc.rounds) <= 1
            orc = O.correct(p.x, p.xb, p.E, p.Delta, k, mu=mu, fixed=True)
        assert rel_err(y, orc.y) <= 1e-5
    ms, mf, nv, ok = O.verify(p.x, y, p.E, p.Delta)
    assert ok and nv == 0
    assert s["max_spatial_err"] == pytest.approx(ms, rel=1e-12)
    assert s["max_spectral_err"] == pytest.approx(mf, rel=1e-8)
    return orc.y


LENGTHS = [2, 3, 7, 8, 64, 100, 1000, 1024, 4096, 4097, 31000, 65536, 100003]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_1d_members_any_length(dt):
    probs = [_member((L,), 100 + i, dt) for i, L in enumerate(LENGTHS)]
    ys, st, stats = _run(probs)
    assert st == F.OK, (st, F.ffcz_last_error(), stats)
    assert all(s["status"] == F.OK for s in stats)
    for p, y, s, L in zip(probs, ys, stats, LENGTHS):
        say(f"[batched] L={L} rounds={s['rounds']}")
        _check(p, y, s, dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_2d_group_mixed_with_1d(dt):
    probs = [_member((64, 128), 200 + i, dt) for i in range(5)]
    probs += [_member((5000,), 300, dt), _member((32, 64), 301, dt), _member((16, 16, 16), 302, dt)]
    ys, st, stats = _run(probs)
    assert st == F.OK, (st, F.ffcz_last_error(), stats)
    for p, y, s in zip(probs, ys, stats):
        _check(p, y, s, dt)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_tiled_1d_passes_match_one_block_bitwise(dt):
    # the same passes split over many blocks per signal: identical bits, counts and maxima
    lengths = [4096, 5000, 31000, 65536, 100003, 131072]
    probs = [_member((L,), 600 + i, dt) for i, L in enumerate(lengths)]
    probs.append(_member((64, 128), 650, dt))  # a 2D group, so the 1D members run beside it
    ys_t, st_t, stats_t = _run(probs, tiled_1d_lg=12)
    ys_b, st_b, stats_b = _run(probs, tiled_1d_lg=21)
    assert st_t == F.OK and st_b == F.OK, (st_t, st_b, F.ffcz_last_error())
    for p, a, b, sa, sb in zip(probs, ys_t, ys_b, stats_t, stats_b):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), p.x.shape
        assert sa == sb, (p.x.shape, sa, sb)
    for p, y, s in zip(probs[:-1], ys_t, stats_t):
        _check(p, y, s, dt)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_lds_resident_1d_matches_memory_bitwise(dt):
    # one block per signal with the work buffer in LDS (FP32 work lengths up to 2^14, FP64 up to
    # 2^13; longer ones keep it in memory) or in the workspace: identical bits, counts and maxima
    lengths = [2, 3, 5, 8, 64, 100, 1000, 1024, 2049, 4096, 4097, 6000, 8192]
    probs = [_member((L,), 700 + i, dt) for i, L in enumerate(lengths)]
    ys_l, st_l, stats_l = _run(probs, resident_1d=True)
    ys_m, st_m, stats_m = _run(probs, resident_1d=False)
    assert st_l == F.OK and st_m == F.OK, (st_l, st_m, F.ffcz_last_error())
    for p, a, b, sa, sb in zip(probs, ys_l, ys_m, stats_l, stats_m):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), p.x.shape
        assert sa == sb, (p.x.shape, sa, sb)
    for p, y, s in zip(probs, ys_l, stats_l):
        _check(p, y, s, dt)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_mixed_batch_graph_and_plain_launches_bitwise(dt):
    # a mixed batch (two 2D groups, tiled and one-block 1D classes): its chunks replayed as one
    # graph with two branches, or launched plainly on two streams, and in chunks of 1 or 4
    # rounds, give identical bits, counts and maxima
    probs = [_member((64, 128), 800 + i, dt) for i in range(3)] + [_member((32, 32), 810, dt)]
    probs += [_member((L,), 820 + i, dt) for i, L in enumerate([3000, 5000, 40000, 70000, 131072])]
    runs = [_run(probs, tiled_1d_lg=14, graph=g, chunk=c) for g, c in ((True, 4), (False, 4), (True, 1))]
    for ys, st, stats in runs:
        assert st == F.OK, (st, F.ffcz_last_error())
    ys0, _, st0 = runs[0]
    for ys, _, stats in runs[1:]:
        for p, a, b, sa, sb in zip(probs, ys0, ys, st0, stats):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), p.x.shape
            assert sa == sb, (p.x.shape, sa, sb)
    for p, y, s in zip(probs, ys0, st0):
        _check(p, y, s, dt)


def test_mixed_batch_fixed_rounds():
    # fixed rounds in a mixed batch: every member runs exactly max_iter projection blocks
    probs = [_member((64, 64), 830 + i, np.float32) for i in range(2)]
    probs += [_member((L,), 840 + i, np.float32) for i, L in enumerate([1000, 9000, 70000])]
    ys, st, stats = _run(probs, max_iter=7, fixed=True, tiled_1d_lg=14)
    assert st == F.OK, (st, F.ffcz_last_error())
    assert [s["rounds"] for s in stats] == [7] * len(probs)
    for p, y, s in zip(probs, ys, stats):
        orc = O.correct(p.x, p.xb, p.E, p.Delta, 7, mu=s["margin_used"], fixed=True)
        assert rel_err(y, orc.y) <= 1e-5


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_batched_matches_single_calls_bitwise(dt):
    # a group of same-shape members and single calls run the same passes (FP64 fields: the
    # closing pass fused with the verification's first pass, over 3 instances or 1)
    import torch
    probs = [_member((64, 128), 400 + i, dt) for i in range(3)]
    ys, st, stats = _run(probs)
    assert st == F.OK, (st, F.ffcz_last_error())
    for p, y, s in zip(probs, ys, stats):
        r = F.correct(torch.from_numpy(p.x).cuda(), torch.from_numpy(p.xb).cuda(), p.E, p.Delta, 200)
        assert np.array_equal(r.y.cpu().numpy().view(np.uint8), y.view(np.uint8))
        assert r.stats["margin_used"] == s["margin_used"]  # same slot rule and fold order
        assert r.stats["max_spatial_err"] == s["max_spatial_err"]
        assert r.stats["max_spectral_err"] == s["max_spectral_err"]


@pytest.mark.parametrize("shape", [(512, 1024), (256, 512)])
def test_batched_tilings(shape):
    # a group of same-shape 2D members (its blocks are numbered across the members): the
    # narrowest tiles (mode 2) give the default tiles' bits; the direct last-axis loop pass
    # (mode 4, 256-entry rows) rounds differently and meets the oracle's bars per member
    probs = [_member(shape, 420 + i, np.float32) for i in range(5)]
    runs = []
    try:
        for mode in (0, 2, 4):
            F.ffcz_set_tuning(mode)
            runs.append(_run(probs))
    finally:
        F.ffcz_set_tuning(1)
    ys0, st0, s0 = runs[0]
    ys2, st2, s2 = runs[1]
    assert st0 == F.OK and st2 == F.OK
    for a, b in zip(ys0, ys2):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert s0 == s2
    ys4, st4, s4 = runs[2]
    assert st4 == F.OK
    for p, y, s in zip(probs, ys4, s4):
        _check(p, y, s, np.float32)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_longest_1d_members(dt):
    # the longest 1D members: 2^19 points (four-step DFT, work length 2^19) and 300007 points
    # (Bluestein, work length 2^20), each against the oracle
    probs = [_member((n,), 600 + i, dt) for i, n in enumerate((1 << 19, 300007))]
    ys, st, stats = _run(probs)
    assert st == F.OK, (st, F.ffcz_last_error(), stats)
    for p, y, s in zip(probs, ys, stats):
        _check(p, y, s, dt)


def test_empty_batch():
    # a batch of no members: a workspace size, then a call that does nothing and succeeds
    import torch
    for dt in (F.F32, F.F64):
        n = F.ffcz_batched_workspace_bytes(dt, [], 10)
        assert n > 0, F.ffcz_last_error()
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        assert F.ffcz_correct_batched(dt, [], 10, None, ws.data_ptr(), n, stream, None) == F.OK
    torch.cuda.synchronize()


def test_batched_statuses():
    # a member capped at 0 rounds reports NOT_CONVERGED; a NaN member reports NONFINITE
    import torch
    a = _member((4096,), 500, np.float32, q=50.0)
    b = _member((64, 64), 501, np.float32, q=50.0)
    ys, st, stats = _run([a, b], max_iter=0)
    assert st == F.NOT_CONVERGED and all(s["rounds"] == 0 for s in stats)
    assert [s["status"] for s in stats] == [F.NOT_CONVERGED, F.NOT_CONVERGED]
    bad = a.xb.copy()
    bad[17] = np.nan
    mem = [(torch.from_numpy(a.x).cuda(), torch.from_numpy(bad).cuda(), a.E, a.Delta)]
    _, st, stats = F.correct_batched(mem, 10, check=False)
    assert st == F.E_NONFINITE and stats[0]["nonfinite"] == 1 and stats[0]["status"] == F.E_NONFINITE


@pytest.mark.timeout(900)
def test_full_batch_eeg_and_diffraction():
    """512 EEG-like signals (lengths log-uniform in [2^12, 2^18]) and 64 diffraction-like
    2048^2 fields in one batched call; every member re-verified in FP64 by the library and by
    torch, and compared with the oracle."""
    import torch
    O.set_workers(max(1, min(16, O.default_workers())))
    say("[full] generating 512 EEG signals and 64 diffraction fields")
    eeg = [W.config_eeg(i) for i in range(512)]
    hedm = [W.config_diffraction(j) for j in range(64)]
    probs = eeg + hedm
    mem = [(torch.from_numpy(p.x).cuda(), torch.from_numpy(p.xb).cuda(), p.E, p.Delta) for p in probs]
    say("[full] batched correction")
    outs, st, stats = F.correct_batched(mem, 200, check=False)
    torch.cuda.synchronize()
    bad = [(i, tuple(probs[i].x.shape), s) for i, s in enumerate(stats) if s["status"] != F.OK]
    for i, shp, s in bad[:8]:
        say(f"[full] member {i} shape {shp} E {probs[i].E:.6g} Delta {probs[i].Delta:.6g}: {s}")
    assert st == max([s["status"] for s in stats] + [F.OK])
    assert st == F.OK and not bad, (st, F.ffcz_last_error(), len(bad))
    for (x, _, E, D), y, s in zip(mem, outs, stats):
        assert s["max_spatial_err"] <= E and s["max_spectral_err"] <= D
        d = y.double() - x.double()
        Dk = torch.fft.rfftn(d)
        assert float(d.abs().max()) <= E
        assert float(torch.maximum(Dk.real.abs().max(), Dk.imag.abs().max())) <= D
    rounds = [s["rounds"] for s in stats]
    say(f"[full] rounds: eeg max {max(rounds[:512])} mean {np.mean(rounds[:512]):.1f}; "
        f"hedm max {max(rounds[512:])} mean {np.mean(rounds[512:]):.1f}")
    # every member against the FP64 oracle
    worst = 0.0
    for i in range(len(probs)):
        if i % 64 == 0:
            say(f"[full] oracle members {i}..{min(i + 63, len(probs) - 1)}")
        y = outs[i].cpu().numpy()
        worst = max(worst, rel_err(y, _check(probs[i], y, stats[i], np.float32)))
    say(f"[full] all {len(probs)} members within {worst:.2e} of the oracle (relative to max|y|)")


def test_batched_reuses_outputs_and_workspace():
    # caller-held outputs and workspace, reused across calls: the same bits as a call that
    # allocates its own; outputs of the wrong shape are refused
    import torch
    probs = [_member((64, 128), 700, np.float32), _member((5000,), 701, np.float32),
             _member((32, 64), 702, np.float32)]
    mem = [(torch.from_numpy(p.x).cuda(), torch.from_numpy(p.xb).cuda(), p.E, p.Delta) for p in probs]
    ref, st0, stats0 = F.correct_batched(mem, 200)
    outs = [torch.empty_like(m[0]) for m in mem]
    ws = F.batched_workspace(mem, 200)
    for _ in range(2):
        got, st, stats = F.correct_batched(mem, 200, ws=ws, outs=outs)
        torch.cuda.synchronize()
        assert st == st0 == F.OK
        assert all(g is o for g, o in zip(got, outs))
        for a, b in zip(ref, got):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32))
        assert stats == stats0
    bad = [torch.empty(3, device="cuda")] + outs[1:]
    with pytest.raises(F.FFCzError):
        F.correct_batched(mem, 200, ws=ws, outs=bad)
