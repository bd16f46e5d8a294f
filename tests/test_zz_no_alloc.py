"""ffcz_correct_noalloc (the entry point that takes its workspace from the library's
fixed device array) against ffcz_correct on the same inputs, through the C ABI:
two calls in a row, the second on a smaller field, in FP32 and FP64."""

import ctypes

import numpy as np
import pytest

from paper_2601_01596_amd import ffcz as F
from paper_2601_01596_amd import workloads as W
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu


def _both(p, dt):
    import torch
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(p.x)).to(dev)
    xb = torch.from_numpy(np.ascontiguousarray(p.xb)).to(dev)
    shape = tuple(x.shape)
    code = F.F32 if dt == np.float32 else F.F64
    stream = torch.cuda.current_stream(dev).cuda_stream
    # the existing entry point with a caller-held workspace
    ws = F.workspace(code, shape, p.max_iter, dev)
    y_ref = torch.empty_like(x)
    st_ref = F.Stats()
    r_ref = F.ffcz_correct(code, shape, x.data_ptr(), xb.data_ptr(), y_ref.data_ptr(), p.E, p.Delta, p.max_iter,
                           None, ws.data_ptr(), ws.numel(), stream, st_ref)
    # the no-allocation entry point
    y = torch.full_like(x, float("nan"))
    st = F.Stats()
    r = F.ffcz_correct_noalloc(code, shape, x.data_ptr(), xb.data_ptr(), y.data_ptr(), p.E, p.Delta, p.max_iter,
                               None, stream, st)
    torch.cuda.synchronize()
    assert r_ref == F.OK, (r_ref, F.ffcz_last_error())
    assert r == F.OK, (r, F.ffcz_last_error())
    return y_ref.cpu().numpy(), y.cpu().numpy(), st_ref, st


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_noalloc_matches_correct_on_two_calls(dt):
    tol = 1e-5 if dt == np.float32 else 1e-12
    # first call 64^3, second call a smaller 32^3 field (the array keeps the first call's
    # contents; the second must not depend on them)
    for n in (64, 32):
        p = W.config_lognormal(n, dt)
        y_ref, y, st_ref, st = _both(p, dt)
        print(f"[noalloc] {np.dtype(dt).name} {n}^3: rounds {st.rounds} / {st_ref.rounds}, "
              f"rel err {rel_err(y, y_ref):.2e}", flush=True)
        assert np.all(np.isfinite(y))
        assert st.rounds == st_ref.rounds and st.converged == st_ref.converged
        assert st.f_viol_initial == st_ref.f_viol_initial and st.s_guard == st_ref.s_guard
        assert rel_err(y, y_ref) <= tol
        assert st.max_spatial_err <= p.E and st.max_spectral_err <= p.Delta
        assert st.max_spatial_err == pytest.approx(st_ref.max_spatial_err, rel=1e-9)


def test_noalloc_refuses_shapes_beyond_its_array():
    # 256^3 FP32 needs far more than the fixed array: refused before any device work
    # (distinct, aligned stand-in addresses that are never dereferenced)
    st = F.ffcz_correct_noalloc(F.F32, (256, 256, 256), 256, 512, 768, 1e-3, 1.0, 10, None, 0, None)
    assert st == F.E_WORKSPACE, F.ffcz_last_error()
    assert "scratch" in F.ffcz_last_error()
    # 1D lengths that take the signal path are refused too
    st = F.ffcz_correct_noalloc(F.F32, (1000,), 256, 512, 768, 1e-3, 1.0, 10, None, 0, None)
    assert st == F.E_SHAPE
