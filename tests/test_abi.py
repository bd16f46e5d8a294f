"""The C-ABI library loads on the CPU and exports every entry point ffcz.h declares.

No compute is called here (no GPU); shape/size queries are host-only."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffcz.h")
LIB = os.path.join(ROOT, "paper_2601_01596_amd", "libffcz.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ffcz_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libffcz.so is not built: run python -m paper_2601_01596_amd.build")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "ffcz_correct" in names and "ffcz_correct_backward" in names
    for n in names:
        assert hasattr(lib, n), n


def test_python_binding_names_match_the_header():
    from paper_2601_01596_amd import ffcz
    for n in declared():
        assert n in ffcz.EXPORTS and callable(getattr(ffcz, n)), n


def test_size_queries_and_shape_rules():
    from paper_2601_01596_amd import ffcz
    assert ffcz.ffcz_version() >= 100
    w = ffcz.ffcz_workspace_bytes(ffcz.F32, (64, 64, 64), 200)
    # two FP32 half-spectra with 128-byte padded rows: 64*64*(33 -> 48) * 8 bytes each
    assert w >= 2 * 64 * 64 * 48 * 8
    assert ffcz.ffcz_workspace_bytes(ffcz.F32, (64, 63, 64), 10) == 0   # not a power of two (3D)
    assert ffcz.ffcz_workspace_bytes(ffcz.F32, (2, 2, 2, 2), 10) == 0   # ndim 4
    assert ffcz.ffcz_workspace_bytes(ffcz.F64, (1, 64, 1), 10) > 0       # squeezes to 1D
    assert ffcz.ffcz_workspace_bytes(ffcz.F32, (0, 64, 64), 10) == 0     # an empty extent
    assert ffcz.ffcz_batched_workspace_bytes(ffcz.F32, [], 10) > 0       # an empty batch
    # masks: (K+1) s-planes of 64*64 rows x 1 word + K f-pairs of 64*64 rows x 1 word
    assert ffcz.ffcz_mask_bytes((64, 64, 64), 3) == 4 * 4096 * 8 + 3 * 2 * 4096 * 8
    assert ffcz.ffcz_mask_bytes((8, 8, 256), 1) == 2 * 64 * 4 * 8 + 2 * 64 * 3 * 8


def test_options_defaults():
    from paper_2601_01596_amd import ffcz
    o = ffcz.ffcz_default_options()
    assert o.verify_fp64 == 1 and o.fixed_iterations == 0 and o.masks_out is None


def test_batched_binding_argument_checks():
    # refused on the host before any device work: host tensors, an outs list of the wrong
    # length, a workspace for no members
    import torch
    from paper_2601_01596_amd import ffcz
    x = torch.zeros(8, 16)
    mem = [(x, x.clone(), 1e-3, 1.0)]
    with pytest.raises(ffcz.FFCzError):
        ffcz.correct_batched(mem, 10)
    with pytest.raises(ffcz.FFCzError):
        ffcz.correct_batched(mem, 10, outs=[])
    with pytest.raises(ffcz.FFCzError):
        ffcz.batched_workspace([], 10)
    assert ffcz.correct_batched([], 10) == ([], ffcz.OK, [])


def test_binding_checks_outputs_masks_and_workspaces():
    # the checks behind correct(out=..., ws=...), correct_backward(masks, ws=...) and
    # correct_batched(ws=..., outs=...), exercised on host tensors: a wrong shape, dtype,
    # device, layout or byte count is refused before any pointer reaches the library
    import torch
    from paper_2601_01596_amd import ffcz
    x = torch.zeros(8, 16)
    ffcz._check_like(torch.empty(8, 16), x, "out")
    for bad in (torch.empty(8, 15), torch.empty(8, 16, dtype=torch.float64), torch.empty(16, 8).t(),
                torch.empty(8, 16, device="meta")):
        with pytest.raises(ffcz.FFCzError):
            ffcz._check_like(bad, x, "out")
    cpu = torch.device("cpu")
    ffcz._check_bytes(torch.empty(100, dtype=torch.uint8), 100, cpu, "ws")
    for bad, n in ((torch.empty(99, dtype=torch.uint8), 100), (torch.empty(100, dtype=torch.float32), 100),
                   (torch.empty(100, dtype=torch.uint8, device="meta"), 100),
                   (torch.empty(200, dtype=torch.uint8)[::2], 100)):
        with pytest.raises(ffcz.FFCzError):
            ffcz._check_bytes(bad, n, cpu, "ws")
    # host tensors are refused by every convenience
    with pytest.raises(ffcz.FFCzError):
        ffcz.correct(x, x.clone(), 1e-3, 1.0, 10)
    with pytest.raises(ffcz.FFCzError):
        ffcz.correct_backward(x, torch.zeros(10, dtype=torch.uint8), 1)


def test_one_dimensional_fields_of_any_length_have_a_workspace():
    # single 1D fields of any length up to 2^19 run on the signal path: a workspace, no masks
    from paper_2601_01596_amd import ffcz
    for L in (1, 3, 4097, 31000, 2 ** 19):
        assert ffcz.ffcz_workspace_bytes(ffcz.F32, (L,), 200) > 0, L
        assert ffcz.ffcz_mask_bytes((L,), 3) == 0
    assert ffcz.ffcz_workspace_bytes(ffcz.F32, (1, 1, 1), 10) > 0
    assert ffcz.ffcz_workspace_bytes(ffcz.F32, (2 ** 19 + 1,), 10) == 0
    assert ffcz.ffcz_mask_bytes((4096,), 3) > 0  # powers of two up to 4096 keep the field passes


def test_strided_copy_argument_checks():
    # refused on the host before any launch, so no GPU is needed
    from paper_2601_01596_amd import ffcz
    E = ffcz.E_INVALID
    assert ffcz.ffcz_copy_columns(0, 0, 4, 4096, 4, 256, 128, 0) == E     # null pointers
    assert ffcz.ffcz_copy_columns(16, 32, -1, 4096, 4, 256, 128, 0) == E  # negative count
    assert ffcz.ffcz_copy_columns(8, 32, 4, 4096, 4, 256, 128, 0) == E    # misaligned pointer
    assert ffcz.ffcz_copy_columns(16, 32, 4, 4100, 4, 256, 128, 0) == E   # misaligned stride
    assert ffcz.ffcz_copy_columns(16, 32, 4, 4096, 4, 256, 120, 0) == E   # row size not 16-byte
    assert ffcz.ffcz_copy_columns(16, 32, 0, 4096, 4, 256, 128, 0) == ffcz.OK  # nothing to copy


def test_profile_select_names():
    from paper_2601_01596_amd import ffcz
    ffcz.ffcz_profile_select(["x_pass", "z_pass"])
    ffcz.ffcz_profile_select(None)
    with pytest.raises(ValueError):
        ffcz.ffcz_profile_select(["no_such_pass"])
