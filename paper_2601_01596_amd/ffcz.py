"""Python binding of ``libffcz.so`` (argument marshalling only).

The functions named ``ffcz_*`` mirror the C ABI of ``include/ffcz.h`` one to
one and take raw device pointers.  ``correct``, ``correct_backward`` and
``FFCzCorrect`` are conveniences over them for torch tensors: torch supplies
device memory and the current stream, every arithmetic step runs in the HIP
library.  There is no fallback: if the library is missing, importing this
module's functions raises.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffcz.so")

F32 = 0
F64 = 1
OK = 0
NOT_CONVERGED = 1
VERIFY_FAILED = 2
E_INVALID = -1
E_SHAPE = -2
E_WORKSPACE = -3
E_NONFINITE = -4
E_HIP = -5

EXPORTS = ("ffcz_version", "ffcz_last_error", "ffcz_default_options", "ffcz_workspace_bytes",
           "ffcz_mask_bytes", "ffcz_suggest_margin", "ffcz_correct", "ffcz_correct_backward",
           "ffcz_batched_workspace_bytes", "ffcz_correct_batched", "ffcz_profile_enable", "ffcz_profile_read",
           "ffcz_profile_select",
           "ffcz_copy", "ffcz_copy_columns", "ffcz_set_tuning", "ffcz_clear_tuning", "ffcz_correct_noalloc",
           "ffcz_default_encode_options", "ffcz_encode_workspace_bytes", "ffcz_encode", "ffcz_decode",
           "ffcz_bounds_workspace_bytes", "ffcz_correct_bounds", "ffcz_power_spectrum_bounds",
           "ffcz_huffman_workspace_bytes", "ffcz_huffman_plan", "ffcz_huffman_encode", "ffcz_huffman_decode")

PROFILE_KINDS = ("init", "y_fwd", "x_pass", "y_inv", "z_pass", "finalize", "verify_z", "verify_y", "verify_x",
                 "adjoint_z", "adjoint_y", "adjoint_x")


class Options(ctypes.Structure):
    _fields_ = [
        ("margin_rel", ctypes.c_double),
        ("fixed_iterations", ctypes.c_int32),
        ("verify_fp64", ctypes.c_int32),
        ("masks_out", ctypes.c_void_p),
        ("viol_per_round", ctypes.c_void_p),
        ("graph_chunk", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("tiled_1d_lg", ctypes.c_int32),
        ("resident_1d", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("f_viol_initial", ctypes.c_int64),
        ("f_viol_final", ctypes.c_int64),
        ("s_clipped_total", ctypes.c_int64),
        ("s_guard", ctypes.c_int64),
        ("nonfinite", ctypes.c_int64),
        ("max_spatial_err", ctypes.c_double),
        ("max_spectral_err", ctypes.c_double),
        ("spectral_viol", ctypes.c_int64),
        ("margin_used", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class HuffmanSizes(ctypes.Structure):
    _fields_ = [
        ("nsym", ctypes.c_int64),
        ("lo", ctypes.c_int64),
        ("nalpha", ctypes.c_int64),
        ("ws_bytes", ctypes.c_size_t),
        ("out_bytes", ctypes.c_size_t),
    ]


class Bounds(ctypes.Structure):
    _fields_ = [
        ("eps_s", ctypes.c_void_p),
        ("delta_re", ctypes.c_void_p),
        ("delta_im", ctypes.c_void_p),
        ("disk", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class EncodeOptions(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("safety", ctypes.c_double),
        ("mu_s", ctypes.c_double),
        ("mu_f", ctypes.c_double),
        ("y_out", ctypes.c_void_p),
        ("spat_edits_out", ctypes.c_void_p),
        ("freq_edits_out", ctypes.c_void_p),
    ]


class EncodeStats(ctypes.Structure):
    _fields_ = [
        ("loop", Stats),
        ("nnz_s", ctypes.c_int64),
        ("nnz_f", ctypes.c_int64),
        ("step_s", ctypes.c_double),
        ("step_f", ctypes.c_double),
        ("mu_s", ctypes.c_double),
        ("mu_f", ctypes.c_double),
        ("m", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


class Instance(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("shape", ctypes.c_int64 * 3),
        ("x_orig", ctypes.c_void_p),
        ("x_base", ctypes.c_void_p),
        ("x_out", ctypes.c_void_p),
        ("eps_s", ctypes.c_double),
        ("delta_f", ctypes.c_double),
    ]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 12), ("count", ctypes.c_int64 * 12)]


class FFCzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ffcz status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libffcz.so`` (built by ``paper_2601_01596_amd.build``); raises if absent.

    torch ships its own HIP runtime under the same sonames as the system's.  It is
    imported first, so the library's ``libamdhip64.so.7`` resolves to the runtime
    torch already loaded: with the library loaded first, torch would bring in a
    second runtime and the library's would see no device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FFCzError(E_HIP, f"{LIB_PATH} is missing: run python -m paper_2601_01596_amd.build")
        try:
            import torch  # noqa: F401
        except ImportError:  # plain C-ABI use without torch: the system runtime
            pass
        L = ctypes.CDLL(LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.ffcz_version.restype = ctypes.c_int32
        L.ffcz_last_error.restype = ctypes.c_char_p
        L.ffcz_default_options.argtypes = [ctypes.POINTER(Options)]
        L.ffcz_default_options.restype = None
        L.ffcz_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_int32]
        L.ffcz_workspace_bytes.restype = ctypes.c_size_t
        L.ffcz_mask_bytes.argtypes = [ctypes.c_int32, i64p, ctypes.c_int32]
        L.ffcz_mask_bytes.restype = ctypes.c_size_t
        L.ffcz_suggest_margin.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double)]
        L.ffcz_suggest_margin.restype = ctypes.c_int32
        L.ffcz_correct.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                   ctypes.POINTER(Stats)]
        L.ffcz_correct.restype = ctypes.c_int32
        L.ffcz_correct_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                           ctypes.POINTER(Options), ctypes.c_void_p, ctypes.POINTER(Stats)]
        L.ffcz_correct_noalloc.restype = ctypes.c_int32
        L.ffcz_default_encode_options.argtypes = [ctypes.POINTER(EncodeOptions)]
        L.ffcz_default_encode_options.restype = None
        L.ffcz_encode_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_int32]
        L.ffcz_encode_workspace_bytes.restype = ctypes.c_size_t
        L.ffcz_encode.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(Options),
                                  ctypes.POINTER(EncodeOptions), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                  ctypes.POINTER(EncodeStats)]
        L.ffcz_encode.restype = ctypes.c_int32
        L.ffcz_decode.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.c_void_p]
        L.ffcz_decode.restype = ctypes.c_int32
        L.ffcz_bounds_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_int32]
        L.ffcz_bounds_workspace_bytes.restype = ctypes.c_size_t
        L.ffcz_correct_bounds.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Bounds),
                                          ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p, ctypes.POINTER(Stats)]
        L.ffcz_correct_bounds.restype = ctypes.c_int32
        L.ffcz_power_spectrum_bounds.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_void_p,
                                                 ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.c_void_p]
        L.ffcz_power_spectrum_bounds.restype = ctypes.c_int32
        L.ffcz_huffman_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
        L.ffcz_huffman_workspace_bytes.restype = ctypes.c_size_t
        L.ffcz_huffman_plan.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(HuffmanSizes)]
        L.ffcz_huffman_plan.restype = ctypes.c_int32
        L.ffcz_huffman_encode.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.POINTER(HuffmanSizes), ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_size_t)]
        L.ffcz_huffman_encode.restype = ctypes.c_int32
        L.ffcz_huffman_decode.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int64)]
        L.ffcz_huffman_decode.restype = ctypes.c_int32
        L.ffcz_correct_backward.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p]
        L.ffcz_correct_backward.restype = ctypes.c_int32
        L.ffcz_batched_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Instance),
                                                   ctypes.c_int32]
        L.ffcz_batched_workspace_bytes.restype = ctypes.c_size_t
        L.ffcz_correct_batched.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Instance), ctypes.c_int32,
                                           ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                           ctypes.POINTER(Stats)]
        L.ffcz_correct_batched.restype = ctypes.c_int32
        L.ffcz_profile_enable.argtypes = [ctypes.c_int32]
        L.ffcz_profile_enable.restype = None
        L.ffcz_profile_read.argtypes = [ctypes.POINTER(Profile)]
        L.ffcz_profile_read.restype = ctypes.c_int32
        L.ffcz_profile_select.argtypes = [ctypes.c_uint32]
        L.ffcz_profile_select.restype = None
        L.ffcz_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ffcz_copy.restype = ctypes.c_int32
        L.ffcz_copy_columns.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int64] * 5 + [ctypes.c_void_p]
        L.ffcz_copy_columns.restype = ctypes.c_int32
        L.ffcz_set_tuning.argtypes = [ctypes.c_int32, ctypes.c_char_p]
        L.ffcz_set_tuning.restype = ctypes.c_int32
        L.ffcz_clear_tuning.argtypes = []
        L.ffcz_clear_tuning.restype = None
        _lib = L
    return _lib


def _shape(shape: Sequence[int]):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return len(shape), arr


# ---------------------------------------------------------------- raw C ABI

def ffcz_version() -> int:
    return lib().ffcz_version()


def ffcz_last_error() -> str:
    return lib().ffcz_last_error().decode()


def ffcz_default_options() -> Options:
    o = Options()
    lib().ffcz_default_options(ctypes.byref(o))
    return o


def ffcz_workspace_bytes(dtype: int, shape: Sequence[int], max_iter: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_workspace_bytes(dtype, nd, arr, max_iter))


def ffcz_mask_bytes(shape: Sequence[int], rounds: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_mask_bytes(nd, arr, rounds))


def ffcz_suggest_margin(dtype: int, shape, x_ptr: int, delta_f: float, ws_ptr: int, ws_bytes: int,
                        stream: int) -> float:
    nd, arr = _shape(shape)
    mu = ctypes.c_double(0.0)
    st = lib().ffcz_suggest_margin(dtype, nd, arr, ctypes.c_void_p(x_ptr), float(delta_f), ctypes.c_void_p(ws_ptr),
                                   ws_bytes, ctypes.c_void_p(stream), ctypes.byref(mu))
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return mu.value


def ffcz_correct(dtype: int, shape, x_ptr: int, xb_ptr: int, y_ptr: int, eps_s: float, delta_f: float,
                 max_iter: int, opts: Optional[Options], ws_ptr: int, ws_bytes: int, stream: int,
                 stats: Optional[Stats]) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_correct(dtype, nd, arr, ctypes.c_void_p(x_ptr), ctypes.c_void_p(xb_ptr),
                                  ctypes.c_void_p(y_ptr), float(eps_s), float(delta_f), int(max_iter),
                                  ctypes.byref(opts) if opts is not None else None, ctypes.c_void_p(ws_ptr),
                                  ws_bytes, ctypes.c_void_p(stream),
                                  ctypes.byref(stats) if stats is not None else None))


def ffcz_correct_noalloc(dtype: int, shape, x_ptr: int, xb_ptr: int, y_ptr: int, eps_s: float, delta_f: float,
                         max_iter: int, opts: Optional[Options], stream: int, stats: Optional[Stats]) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_correct_noalloc(dtype, nd, arr, ctypes.c_void_p(x_ptr), ctypes.c_void_p(xb_ptr),
                                          ctypes.c_void_p(y_ptr), float(eps_s), float(delta_f), int(max_iter),
                                          ctypes.byref(opts) if opts is not None else None,
                                          ctypes.c_void_p(stream), ctypes.byref(stats) if stats is not None else None))


def ffcz_bounds_workspace_bytes(dtype: int, shape: Sequence[int], max_iter: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_bounds_workspace_bytes(dtype, nd, arr, max_iter))


def ffcz_correct_bounds(dtype: int, shape, x_ptr: int, xb_ptr: int, y_ptr: int, eps_s: float, delta_f: float,
                        bounds: Optional[Bounds], max_iter: int, opts: Optional[Options], ws_ptr: int, ws_bytes: int,
                        stream: int, stats: Optional[Stats]) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_correct_bounds(dtype, nd, arr, ctypes.c_void_p(x_ptr), ctypes.c_void_p(xb_ptr),
                                         ctypes.c_void_p(y_ptr), float(eps_s), float(delta_f),
                                         ctypes.byref(bounds) if bounds is not None else None, int(max_iter),
                                         ctypes.byref(opts) if opts is not None else None, ctypes.c_void_p(ws_ptr),
                                         ws_bytes, ctypes.c_void_p(stream),
                                         ctypes.byref(stats) if stats is not None else None))


def ffcz_power_spectrum_bounds(dtype: int, shape, x_ptr: int, rho: float, disk: int, out_ptr: int, ws_ptr: int,
                               ws_bytes: int, stream: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_power_spectrum_bounds(dtype, nd, arr, ctypes.c_void_p(x_ptr), float(rho), int(disk),
                                                ctypes.c_void_p(out_ptr), ctypes.c_void_p(ws_ptr), ws_bytes,
                                                ctypes.c_void_p(stream)))


def ffcz_huffman_workspace_bytes(nsym: int, nalpha: int) -> int:
    return int(lib().ffcz_huffman_workspace_bytes(int(nsym), int(nalpha)))


def ffcz_huffman_plan(sym_ptr: int, nsym: int, width: int, ws_ptr: int, ws_bytes: int, stream: int,
                      sizes: HuffmanSizes) -> int:
    return int(lib().ffcz_huffman_plan(ctypes.c_void_p(sym_ptr), int(nsym), int(width), ctypes.c_void_p(ws_ptr),
                                       ws_bytes, ctypes.c_void_p(stream), ctypes.byref(sizes)))


def ffcz_huffman_encode(sym_ptr: int, nsym: int, width: int, sizes: HuffmanSizes, out_ptr: int, out_bytes: int,
                        ws_ptr: int, ws_bytes: int, stream: int):
    used = ctypes.c_size_t(0)
    st = int(lib().ffcz_huffman_encode(ctypes.c_void_p(sym_ptr), int(nsym), int(width), ctypes.byref(sizes),
                                       ctypes.c_void_p(out_ptr), out_bytes, ctypes.c_void_p(ws_ptr), ws_bytes,
                                       ctypes.c_void_p(stream), ctypes.byref(used)))
    return st, int(used.value)


def ffcz_huffman_decode(in_ptr: int, in_bytes: int, width: int, out_ptr: int, capacity: int, ws_ptr: int,
                        ws_bytes: int, stream: int):
    n = ctypes.c_int64(0)
    st = int(lib().ffcz_huffman_decode(ctypes.c_void_p(in_ptr), in_bytes, int(width), ctypes.c_void_p(out_ptr),
                                       int(capacity), ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream),
                                       ctypes.byref(n)))
    return st, int(n.value)


def ffcz_default_encode_options() -> EncodeOptions:
    o = EncodeOptions()
    lib().ffcz_default_encode_options(ctypes.byref(o))
    return o


def ffcz_encode_workspace_bytes(dtype: int, shape: Sequence[int], max_iter: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_encode_workspace_bytes(dtype, nd, arr, max_iter))


def ffcz_encode(dtype: int, shape, x_ptr: int, xb_ptr: int, eps_s: float, delta_f: float, max_iter: int,
                opts: Optional[Options], eopts: Optional[EncodeOptions], sflags_ptr: int, scodes_ptr: int,
                fflags_ptr: int, fcodes_ptr: int, ws_ptr: int, ws_bytes: int, stream: int,
                stats: Optional[EncodeStats]) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_encode(dtype, nd, arr, ctypes.c_void_p(x_ptr), ctypes.c_void_p(xb_ptr), float(eps_s),
                                 float(delta_f), int(max_iter), ctypes.byref(opts) if opts is not None else None,
                                 ctypes.byref(eopts) if eopts is not None else None, ctypes.c_void_p(sflags_ptr),
                                 ctypes.c_void_p(scodes_ptr), ctypes.c_void_p(fflags_ptr),
                                 ctypes.c_void_p(fcodes_ptr), ctypes.c_void_p(ws_ptr), ws_bytes,
                                 ctypes.c_void_p(stream), ctypes.byref(stats) if stats is not None else None))


def ffcz_decode(dtype: int, shape, xb_ptr: int, sflags_ptr: int, scodes_ptr: int, nnz_s: int, fflags_ptr: int,
                fcodes_ptr: int, nnz_f: int, step_s: float, step_f: float, y_ptr: int, ws_ptr: int, ws_bytes: int,
                stream: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_decode(dtype, nd, arr, ctypes.c_void_p(xb_ptr), ctypes.c_void_p(sflags_ptr),
                                 ctypes.c_void_p(scodes_ptr), int(nnz_s), ctypes.c_void_p(fflags_ptr),
                                 ctypes.c_void_p(fcodes_ptr), int(nnz_f), float(step_s), float(step_f),
                                 ctypes.c_void_p(y_ptr), ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream)))


def ffcz_correct_backward(dtype: int, shape, rounds: int, masks_ptr: int, grad_out_ptr: int, grad_base_ptr: int,
                          ws_ptr: int, ws_bytes: int, stream: int) -> int:
    nd, arr = _shape(shape)
    return int(lib().ffcz_correct_backward(dtype, nd, arr, int(rounds), ctypes.c_void_p(masks_ptr),
                                           ctypes.c_void_p(grad_out_ptr), ctypes.c_void_p(grad_base_ptr),
                                           ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream)))


def ffcz_batched_workspace_bytes(dtype: int, instances, max_iter: int) -> int:
    arr = (Instance * len(instances))(*instances)
    return int(lib().ffcz_batched_workspace_bytes(dtype, len(instances), arr, max_iter))


def ffcz_correct_batched(dtype: int, instances, max_iter: int, opts: Optional[Options], ws_ptr: int, ws_bytes: int,
                         stream: int, stats) -> int:
    arr = (Instance * len(instances))(*instances)
    return int(lib().ffcz_correct_batched(dtype, len(instances), arr, int(max_iter),
                                          ctypes.byref(opts) if opts is not None else None, ctypes.c_void_p(ws_ptr),
                                          ws_bytes, ctypes.c_void_p(stream), stats))


def ffcz_profile_enable(on: bool) -> None:
    lib().ffcz_profile_enable(1 if on else 0)


def ffcz_profile_select(kinds=None) -> None:
    """Time only the named pass kinds (names from PROFILE_KINDS); None times every kind."""
    mask = 0
    for k in (kinds or ()):
        mask |= 1 << PROFILE_KINDS.index(k)
    lib().ffcz_profile_select(mask)


def ffcz_profile_read() -> dict:
    """Summed device ms and launch counts per pass kind since the last read."""
    pr = Profile()
    st = lib().ffcz_profile_read(ctypes.byref(pr))
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return {k: (pr.ms[i], int(pr.count[i])) for i, k in enumerate(PROFILE_KINDS)}


def ffcz_set_tuning(mode: int, cache_path=None) -> int:
    """Tile tuning mode (0 default tiles, 1 tune on first use, 2 narrowest) and cache file."""
    p = None if cache_path is None else str(cache_path).encode()
    return int(lib().ffcz_set_tuning(int(mode), p))


def ffcz_clear_tuning() -> None:
    lib().ffcz_clear_tuning()


def ffcz_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int) -> int:
    return int(lib().ffcz_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nbytes),
                               ctypes.c_void_p(stream)))


# ---------------------------------------------------------------- torch conveniences

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise FFCzError(E_INVALID, f"unsupported dtype {t.dtype}")


def _check_tensor(t, name):
    if not t.is_cuda:
        raise FFCzError(E_INVALID, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise FFCzError(E_INVALID, f"{name} must be contiguous")


def _check_like(t, ref, name):
    """``t`` must be a contiguous tensor of ``ref``'s shape, dtype and device (a wrong
    size would let the kernels write past it)."""
    if not t.is_contiguous():
        raise FFCzError(E_INVALID, f"{name} must be contiguous")
    if tuple(t.shape) != tuple(ref.shape) or t.dtype != ref.dtype or t.device != ref.device:
        raise FFCzError(E_INVALID, f"{name} must match shape {tuple(ref.shape)}, dtype {ref.dtype} and "
                                   f"device {ref.device}")


def _check_bytes(t, nbytes: int, device, name):
    """``t`` must be a contiguous uint8 device tensor on ``device`` of at least ``nbytes`` bytes."""
    torch = _torch()
    if not t.is_contiguous():
        raise FFCzError(E_INVALID, f"{name} must be contiguous")
    if t.dtype != torch.uint8 or t.device != device:
        raise FFCzError(E_INVALID, f"{name} must be a uint8 tensor on {device}")
    if t.numel() < nbytes:
        raise FFCzError(E_WORKSPACE, f"{name} holds {t.numel()} bytes, {nbytes} needed")


def copy_(dst, src):
    """dst[:] = src with the library's streaming copy kernel, on the current stream."""
    torch = _torch()
    if dst.numel() * dst.element_size() != src.numel() * src.element_size():
        raise ValueError("copy_: byte sizes differ")
    if not (dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("copy_: tensors must be contiguous")
    st = ffcz_copy(dst.data_ptr(), src.data_ptr(), src.numel() * src.element_size(),
                   torch.cuda.current_stream(src.device).cuda_stream)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return dst


def ffcz_copy_columns(dst_ptr: int, src_ptr: int, n_axis: int, axis_stride: int, n_fixed: int,
                      fixed_stride: int, row_bytes: int, stream: int) -> int:
    return int(lib().ffcz_copy_columns(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(n_axis),
                                       int(axis_stride), int(n_fixed), int(fixed_stride), int(row_bytes),
                                       ctypes.c_void_p(stream)))


def copy_columns_(dst, src, n_axis: int, axis_stride: int, n_fixed: int, fixed_stride: int, row_bytes: int):
    """Rows (f, i) of row_bytes bytes at f * fixed_stride + i * axis_stride copied from src to dst
    (contiguous device tensors, viewed as bytes) with the strided passes' access pattern, on the
    current stream."""
    torch = _torch()
    if not (dst.is_contiguous() and src.is_contiguous()) or dst.device != src.device or not src.is_cuda:
        raise ValueError("copy_columns_: contiguous device tensors on one device")
    if min(n_axis, n_fixed, row_bytes, axis_stride, fixed_stride) < 0:
        raise ValueError("copy_columns_: negative argument")
    if n_axis and n_fixed and row_bytes:
        need = (n_fixed - 1) * fixed_stride + (n_axis - 1) * axis_stride + row_bytes
        for t, name in ((dst, "dst"), (src, "src")):
            if t.numel() * t.element_size() < need:
                raise ValueError(f"copy_columns_: {name} holds fewer than the {need} bytes the rows reach")
    st = ffcz_copy_columns(dst.data_ptr(), src.data_ptr(), n_axis, axis_stride, n_fixed, fixed_stride, row_bytes,
                           torch.cuda.current_stream(src.device).cuda_stream)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return dst


def workspace(dtype_code: int, shape, max_iter: int, device=None):
    torch = _torch()
    nbytes = ffcz_workspace_bytes(dtype_code, shape, max_iter)
    if nbytes == 0:
        raise FFCzError(E_SHAPE, f"unsupported shape {tuple(shape)}: {ffcz_last_error()}")
    # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


@dataclasses.dataclass
class Result:
    y: object
    status: int
    stats: dict
    masks: object = None
    viol: object = None


def correct(x, xb, eps_s: float, delta_f: float, max_iter: int, *, margin: float = 0.0, fixed: bool = False,
            verify: bool = True, record_masks: bool = False, record_viol: bool = False, chunk: int = 4,
            graph: bool = True, out=None, ws=None, check: bool = True) -> Result:
    """Run ``ffcz_correct`` on device tensors ``x`` (original) and ``xb`` (base)."""
    torch = _torch()
    _check_tensor(x, "x")
    _check_tensor(xb, "xb")
    if x.shape != xb.shape or x.dtype != xb.dtype:
        raise FFCzError(E_INVALID, "x and xb must have the same shape and dtype")
    if x.device != xb.device:
        raise FFCzError(E_INVALID, "x and xb must be on one device")
    dt = _dtype_code(x)
    shape = tuple(x.shape)
    if out is None:
        y = torch.empty_like(x)
    else:
        _check_like(out, x, "out")
        y = out
    if ws is None:
        ws = workspace(dt, shape, max_iter, x.device)
    else:
        _check_bytes(ws, ffcz_workspace_bytes(dt, shape, max_iter), x.device, "ws")
    opts = ffcz_default_options()
    opts.margin_rel = float(margin)
    opts.fixed_iterations = 1 if fixed else 0
    opts.verify_fp64 = 1 if verify else 0
    opts.graph_chunk = int(chunk)
    opts.use_graph = 1 if graph else 0
    masks = None
    if record_masks:
        nb = ffcz_mask_bytes(shape, max_iter)
        if nb == 0:
            raise FFCzError(E_SHAPE, f"no masks are recorded for shape {shape}")
        masks = torch.zeros(nb, dtype=torch.uint8, device=x.device)
        opts.masks_out = masks.data_ptr()
    viol = None
    if record_viol:
        viol = torch.zeros(max_iter + 1, dtype=torch.int64, device=x.device)
        opts.viol_per_round = viol.data_ptr()
    stats = Stats()
    stream = torch.cuda.current_stream(x.device).cuda_stream
    st = ffcz_correct(dt, shape, x.data_ptr(), xb.data_ptr(), y.data_ptr(), eps_s, delta_f, max_iter, opts,
                      ws.data_ptr(), ws.numel(), stream, stats)
    if check and st < 0:
        raise FFCzError(st, ffcz_last_error())
    return Result(y=y, status=st, stats=stats.as_dict(), masks=masks, viol=viol)


def _squeezed(shape):
    s = tuple(int(n) for n in shape if int(n) > 1)
    return s if s else (1,)


def edit_coords(shape):
    """(spatial, frequency) coordinate counts of the edit coding: N and 2 M, with M the
    half-spectrum entries of the squeezed shape."""
    sq = _squeezed(shape)
    n = 1
    for v in sq:
        n *= v
    m = n // sq[-1] * (sq[-1] // 2 + 1)
    return n, 2 * m


@dataclasses.dataclass
class Encoded:
    """Output of ``encode``: flags (uint8) and codes (int32, trimmed to their counts) of both
    edit sets, the steps, the shrinks and the loop statistics."""
    shape: tuple
    dtype: int
    spat_flags: object
    spat_codes: object
    freq_flags: object
    freq_codes: object
    step_s: float
    step_f: float
    mu_s: float
    mu_f: float
    m: int
    status: int
    stats: dict
    y: object = None
    spat_edits: object = None
    freq_edits: object = None


def encode(x, xb, eps_s: float, delta_f: float, max_iter: int, *, m: int = 16, safety: float = 4.0,
           mus=None, want_y: bool = False, export_edits: bool = False, verify: bool = True, chunk: int = 4,
           graph: bool = True, ws=None, check: bool = True) -> Encoded:
    """``ffcz_encode`` on device tensors: the loop with edit bookkeeping, then flags and codes."""
    torch = _torch()
    _check_tensor(x, "x")
    _check_tensor(xb, "xb")
    if x.shape != xb.shape or x.dtype != xb.dtype or x.device != xb.device:
        raise FFCzError(E_INVALID, "x and xb must have the same shape, dtype and device")
    dt = _dtype_code(x)
    shape = tuple(x.shape)
    ns, nf = edit_coords(shape)
    dev = x.device
    nbytes = ffcz_encode_workspace_bytes(dt, shape, max_iter)
    if nbytes == 0:
        raise FFCzError(E_SHAPE, f"unsupported shape {shape}: {ffcz_last_error()}")
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    else:
        _check_bytes(ws, nbytes, dev, "ws")
    # flag buffers rounded up to 16 bytes (the kernels write whole 8-byte words where they fit)
    sflags = torch.zeros(((ns + 7) // 8 + 15) // 16 * 16, dtype=torch.uint8, device=dev)
    fflags = torch.zeros(((nf + 7) // 8 + 15) // 16 * 16, dtype=torch.uint8, device=dev)
    scodes = torch.empty(max(ns, 1), dtype=torch.int32, device=dev)
    fcodes = torch.empty(max(nf, 1), dtype=torch.int32, device=dev)
    eo = ffcz_default_encode_options()
    eo.m = int(m)
    eo.safety = float(safety)
    if mus is not None:
        eo.mu_s, eo.mu_f = float(mus[0]), float(mus[1])
    y = se = fe = None
    if want_y:
        y = torch.empty_like(x)
        eo.y_out = y.data_ptr()
    if export_edits:
        se = torch.empty(ns, dtype=x.dtype, device=dev)
        fe = torch.empty(nf, dtype=x.dtype, device=dev)
        eo.spat_edits_out = se.data_ptr()
        eo.freq_edits_out = fe.data_ptr()
    opts = ffcz_default_options()
    opts.verify_fp64 = 1 if verify else 0
    opts.graph_chunk = int(chunk)
    opts.use_graph = 1 if graph else 0
    st = EncodeStats()
    stream = torch.cuda.current_stream(dev).cuda_stream
    r = ffcz_encode(dt, shape, x.data_ptr(), xb.data_ptr(), eps_s, delta_f, max_iter, opts, eo, sflags.data_ptr(),
                    scodes.data_ptr(), fflags.data_ptr(), fcodes.data_ptr(), ws.data_ptr(), ws.numel(), stream, st)
    if check and r < 0:
        raise FFCzError(r, ffcz_last_error())
    nbs, nbf = (ns + 7) // 8, (nf + 7) // 8
    return Encoded(shape=shape, dtype=dt, spat_flags=sflags[:nbs], spat_codes=scodes[:st.nnz_s],
                   freq_flags=fflags[:nbf], freq_codes=fcodes[:st.nnz_f], step_s=st.step_s, step_f=st.step_f,
                   mu_s=st.mu_s, mu_f=st.mu_f, m=st.m, status=r, stats=st.loop.as_dict(), y=y, spat_edits=se,
                   freq_edits=fe)


def decode(xb, enc: Encoded, *, ws=None, out=None):
    """``ffcz_decode``: ``y = x_hat + s + IFFT(f)`` from an ``Encoded`` (device tensors)."""
    torch = _torch()
    _check_tensor(xb, "xb")
    dt = _dtype_code(xb)
    shape = tuple(xb.shape)
    if shape != tuple(enc.shape) or dt != enc.dtype:
        raise FFCzError(E_INVALID, "x_hat does not match the encoding's shape and dtype")
    dev = xb.device
    nbytes = ffcz_encode_workspace_bytes(dt, shape, 0)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    else:
        _check_bytes(ws, nbytes, dev, "ws")
    if out is None:
        y = torch.empty_like(xb)
    else:
        _check_like(out, xb, "out")
        y = out

    def aligned(t):
        # the C ABI wants 16-byte aligned buffers (the encoder's slices start at their base)
        t = t.contiguous()
        if t.data_ptr() % 16:
            t = t.clone()
        return t

    sf, ff = aligned(enc.spat_flags), aligned(enc.freq_flags)
    sc, fc = aligned(enc.spat_codes), aligned(enc.freq_codes)
    stream = torch.cuda.current_stream(dev).cuda_stream
    r = ffcz_decode(dt, shape, xb.data_ptr(), sf.data_ptr(), sc.data_ptr() if sc.numel() else 0, sc.numel(),
                    ff.data_ptr(), fc.data_ptr() if fc.numel() else 0, fc.numel(), enc.step_s, enc.step_f,
                    y.data_ptr(), ws.data_ptr(), ws.numel(), stream)
    if r < 0:
        raise FFCzError(r, ffcz_last_error())
    return y


def half_shape(shape):
    """Half-spectrum shape of a field (last axis n -> n // 2 + 1)."""
    shape = tuple(int(n) for n in shape)
    return shape[:-1] + (shape[-1] // 2 + 1,)


def correct_bounds(x, xb, max_iter: int, *, eps_s: float = 0.0, delta_f: float = 0.0, E=None, D_re=None,
                   D_im=None, disk: bool = False, margin: float = 0.0, fixed: bool = False, verify: bool = True,
                   chunk: int = 4, graph: bool = True, out=None, ws=None, check: bool = True) -> Result:
    """``ffcz_correct_bounds`` on device tensors: pointwise bound tensors ``E`` (shape of x),
    ``D_re`` / ``D_im`` (half-spectrum shape), or the scalars where a tensor is None."""
    torch = _torch()
    _check_tensor(x, "x")
    _check_tensor(xb, "xb")
    if x.shape != xb.shape or x.dtype != xb.dtype or x.device != xb.device:
        raise FFCzError(E_INVALID, "x and xb must have the same shape, dtype and device")
    dt = _dtype_code(x)
    shape = tuple(x.shape)
    b = Bounds()
    b.disk = 1 if disk else 0
    keep = []
    for name, t, shp in (("eps_s", E, shape), ("delta_re", D_re, half_shape(shape)),
                         ("delta_im", D_im, half_shape(shape))):
        if t is None:
            continue
        if tuple(t.shape) != tuple(shp) or t.dtype != x.dtype or t.device != x.device or not t.is_contiguous():
            raise FFCzError(E_INVALID, f"{name} must be a contiguous {x.dtype} tensor of shape {shp} on {x.device}")
        keep.append(t)
        setattr(b, name, t.data_ptr())
    y = torch.empty_like(x) if out is None else out
    if out is not None:
        _check_like(out, x, "out")
    nbytes = ffcz_bounds_workspace_bytes(dt, shape, max_iter)
    if nbytes == 0:
        raise FFCzError(E_SHAPE, f"unsupported shape {shape}: {ffcz_last_error()}")
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    else:
        _check_bytes(ws, nbytes, x.device, "ws")
    opts = ffcz_default_options()
    opts.margin_rel = float(margin)
    opts.fixed_iterations = 1 if fixed else 0
    opts.verify_fp64 = 1 if verify else 0
    opts.graph_chunk = int(chunk)
    opts.use_graph = 1 if graph else 0
    stats = Stats()
    stream = torch.cuda.current_stream(x.device).cuda_stream
    st = ffcz_correct_bounds(dt, shape, x.data_ptr(), xb.data_ptr(), y.data_ptr(), eps_s, delta_f, b, max_iter, opts,
                             ws.data_ptr(), ws.numel(), stream, stats)
    if check and st < 0:
        raise FFCzError(st, ffcz_last_error())
    return Result(y=y, status=st, stats=stats.as_dict())


def power_spectrum_bounds(x, rho: float, *, disk: bool = False, ws=None):
    """``ffcz_power_spectrum_bounds``: the half-spectrum bound tensor that keeps every shell of
    the power spectrum of ``x`` within ``rho`` relative error."""
    torch = _torch()
    _check_tensor(x, "x")
    dt = _dtype_code(x)
    shape = tuple(x.shape)
    nbytes = ffcz_bounds_workspace_bytes(dt, shape, 0)
    if nbytes == 0:
        raise FFCzError(E_SHAPE, f"unsupported shape {shape}: {ffcz_last_error()}")
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    else:
        _check_bytes(ws, nbytes, x.device, "ws")
    out = torch.empty(half_shape(shape), dtype=x.dtype, device=x.device)
    st = ffcz_power_spectrum_bounds(dt, shape, x.data_ptr(), rho, 1 if disk else 0, out.data_ptr(), ws.data_ptr(),
                                    ws.numel(), torch.cuda.current_stream(x.device).cuda_stream)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return out


def huffman_compress(sym):
    """Huffman-code a device tensor of symbols (uint8: width 1; int32: width 4).  Returns
    ``(stream uint8 tensor, HuffmanSizes)``."""
    torch = _torch()
    _check_tensor(sym, "sym")
    if sym.dtype == torch.uint8:
        width = 1
    elif sym.dtype == torch.int32:
        width = 4
    else:
        raise FFCzError(E_INVALID, "symbols must be uint8 or int32")
    n = sym.numel()
    stream = torch.cuda.current_stream(sym.device).cuda_stream
    ws = torch.empty(max(ffcz_huffman_workspace_bytes(n, 0), 256), dtype=torch.uint8, device=sym.device)
    sizes = HuffmanSizes()
    st = ffcz_huffman_plan(sym.data_ptr(), n, width, ws.data_ptr(), ws.numel(), stream, sizes)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    ws = torch.empty(max(int(sizes.ws_bytes), 256), dtype=torch.uint8, device=sym.device)
    out = torch.empty(int(sizes.out_bytes), dtype=torch.uint8, device=sym.device)
    st, used = ffcz_huffman_encode(sym.data_ptr(), n, width, sizes, out.data_ptr(), out.numel(), ws.data_ptr(),
                                   ws.numel(), stream)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return out[:used], sizes


def huffman_decompress(stream_t, n: int, dtype, nalpha: int):
    """Decode a stream of ``n`` symbols (``dtype`` uint8 or int32) from ``huffman_compress``."""
    torch = _torch()
    width = 1 if dtype == torch.uint8 else 4
    ws = torch.empty(max(ffcz_huffman_workspace_bytes(n, nalpha), 256), dtype=torch.uint8, device=stream_t.device)
    out = torch.empty(max(n, 1), dtype=dtype, device=stream_t.device)
    st, m = ffcz_huffman_decode(stream_t.data_ptr(), stream_t.numel(), width, out.data_ptr(), out.numel(),
                                ws.data_ptr(), ws.numel(), torch.cuda.current_stream(stream_t.device).cuda_stream)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return out[:m]


def batched_workspace(members, max_iter: int, device=None):
    """A workspace of ``ffcz_batched_workspace_bytes`` bytes for ``members`` (only their
    shapes and dtype count), for reuse across ``correct_batched`` calls."""
    torch = _torch()
    if not members:
        raise FFCzError(E_INVALID, "no members")
    dt = _dtype_code(members[0][0])
    insts = []
    for m in members:
        x = m[0]
        sh = list(x.shape) + [1] * (3 - x.dim())
        insts.append(Instance(x.dim(), 0, (ctypes.c_int64 * 3)(*sh), 0, 0, 0, 0.0, 0.0))
    nbytes = ffcz_batched_workspace_bytes(dt, insts, max_iter)
    if nbytes == 0:
        raise FFCzError(E_SHAPE, ffcz_last_error())
    return torch.empty(nbytes, dtype=torch.uint8, device=device if device is not None else members[0][0].device)


def correct_batched(members, max_iter: int, *, margin: float = 0.0, fixed: bool = False, verify: bool = True,
                    chunk: int = 4, graph: bool = True, tiled_1d_lg: int = 0, resident_1d: bool = True, ws=None,
                    check: bool = True, outs=None):
    """``ffcz_correct_batched`` over ``members = [(x, xb, eps_s, delta_f), ...]`` (device tensors).

    ``outs``: optional output tensors, one per member (same shape and dtype as its x);
    allocated here when omitted.  Returns ``(outputs, status, per-member stats dicts)``.
    """
    torch = _torch()
    if not members:
        return [], OK, []
    if outs is not None and len(outs) != len(members):
        raise FFCzError(E_INVALID, "outs must hold one tensor per member")
    dt = _dtype_code(members[0][0])
    insts = []
    given = outs
    outs = []
    for i, (x, xb, E, D) in enumerate(members):
        _check_tensor(x, "x")
        _check_tensor(xb, "xb")
        if x.shape != xb.shape or x.dtype != xb.dtype or _dtype_code(x) != dt:
            raise FFCzError(E_INVALID, "members must pair tensors of one dtype")
        if x.dim() < 1 or x.dim() > 3:
            raise FFCzError(E_SHAPE, "members must have 1 to 3 dimensions")
        if given is None:
            y = torch.empty_like(x)
        else:
            y = given[i]
            _check_like(y, x, "out")
        outs.append(y)
        sh = list(x.shape) + [1] * (3 - x.dim())
        insts.append(Instance(x.dim(), 0, (ctypes.c_int64 * 3)(*sh), x.data_ptr(), xb.data_ptr(), y.data_ptr(),
                              float(E), float(D)))
    dev = members[0][0].device
    for x, xb, _, _ in members:
        if x.device != dev or xb.device != dev:
            raise FFCzError(E_INVALID, "every member must be on one device")
    nbytes = ffcz_batched_workspace_bytes(dt, insts, max_iter)
    if nbytes == 0:
        raise FFCzError(E_SHAPE, ffcz_last_error())
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    else:
        _check_bytes(ws, nbytes, dev, "ws")
    opts = ffcz_default_options()
    opts.margin_rel = float(margin)
    opts.fixed_iterations = 1 if fixed else 0
    opts.verify_fp64 = 1 if verify else 0
    opts.graph_chunk = int(chunk)
    opts.use_graph = 1 if graph else 0
    if tiled_1d_lg:
        opts.tiled_1d_lg = int(tiled_1d_lg)
    opts.resident_1d = 1 if resident_1d else 0
    stats = (Stats * len(insts))()
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = ffcz_correct_batched(dt, insts, max_iter, opts, ws.data_ptr(), ws.numel(), stream, stats)
    if check and st < 0:
        raise FFCzError(st, ffcz_last_error())
    return outs, st, [s.as_dict() for s in stats]


def correct_backward(grad_y, masks, rounds: int, ws=None):
    """``ffcz_correct_backward``: dL/dx_hat from dL/dy and the recorded masks."""
    torch = _torch()
    _check_tensor(grad_y, "grad_y")
    dt = _dtype_code(grad_y)
    shape = tuple(grad_y.shape)
    nb = ffcz_mask_bytes(shape, rounds)
    if nb == 0:
        raise FFCzError(E_SHAPE, f"no masks exist for shape {shape} and {rounds} rounds")
    _check_bytes(masks, nb, grad_y.device, "masks")
    if ws is None:
        ws = workspace(dt, shape, rounds, grad_y.device)
    else:
        _check_bytes(ws, ffcz_workspace_bytes(dt, shape, rounds), grad_y.device, "ws")
    gb = torch.empty_like(grad_y)
    stream = torch.cuda.current_stream(grad_y.device).cuda_stream
    st = ffcz_correct_backward(dt, shape, rounds, masks.data_ptr(), grad_y.data_ptr(), gb.data_ptr(),
                               ws.data_ptr(), ws.numel(), stream)
    if st < 0:
        raise FFCzError(st, ffcz_last_error())
    return gb


def _autograd():
    torch = _torch()

    class FFCzCorrect(torch.autograd.Function):
        """``y = FFCzCorrect.apply(xb, x, eps_s, delta_f, K)``: K fixed rounds, differentiable in xb.

        The forward records 1-bit clip masks per round; the backward replays the
        rounds in reverse with masks in place of clips (no stored iterates).
        Since ``y = x + eps_K(x_hat - x)``, the gradient with respect to ``x`` is
        ``dL/dy - dL/dx_hat`` (returned when ``x`` requires it).
        """

        @staticmethod
        def forward(ctx, xb, x, eps_s, delta_f, K, margin=0.0):
            r = correct(x.detach(), xb.detach(), eps_s, delta_f, int(K), margin=margin, fixed=True,
                        verify=False, record_masks=True)
            ctx.save_for_backward(r.masks)
            ctx.K = int(K)
            return r.y

        @staticmethod
        def backward(ctx, gy):
            (masks,) = ctx.saved_tensors
            gy = gy.contiguous()
            gb = correct_backward(gy, masks, ctx.K)
            gx = gy - gb if ctx.needs_input_grad[1] else None
            return gb, gx, None, None, None, None

    return FFCzCorrect


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _autograd()
        return getattr(_Lazy._cls, name)


FFCzCorrect = _Lazy()
