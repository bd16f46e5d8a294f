"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
unpack its outputs for comparison with the oracle."""

import numpy as np

from paper_2601_01596_amd import ffcz as F


def cuda_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


def run_gpu(x, xb, E, D, max_iter, **kw):
    """Upload, run ffcz_correct, return (y numpy, Result)."""
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    bt = torch.from_numpy(np.ascontiguousarray(xb)).cuda()
    r = F.correct(xt, bt, E, D, max_iter, check=False, **kw)
    torch.cuda.synchronize()
    return r.y.cpu().numpy(), r


def squeezed(shape):
    s = tuple(n for n in shape if n > 1)
    return s if s else (1,)


def unpack_masks(masks_u8, shape, rounds):
    """Split the ffcz_mask_bytes() record into the oracle's Masks layout (bool arrays)."""
    from oracle.ffcz import Masks
    sh = squeezed(shape)
    nl = sh[-1]
    rows = int(np.prod(sh)) // nl
    hc = nl // 2 + 1
    sw = (nl + 63) // 64
    fw = (hc + 63) // 64
    b = np.asarray(masks_u8, dtype=np.uint8)
    s_plane = rows * sw * 8
    f_plane = rows * fw * 8

    def plane(off, words, n, outshape):
        raw = b[off: off + rows * words * 8].reshape(rows, words * 8)
        bits = np.unpackbits(raw, axis=1, bitorder="little")[:, :n]
        return bits.astype(bool).reshape(outshape)

    hshape = sh[:-1] + (hc,)
    s = [plane(k * s_plane, sw, nl, shape) for k in range(rounds + 1)]
    base = (rounds + 1) * s_plane
    fre = [None]
    fim = [None]
    full_h = tuple(shape[:-1]) + (shape[-1] // 2 + 1,)
    for k in range(1, rounds + 1):
        o = base + (k - 1) * 2 * f_plane
        fre.append(plane(o, fw, hc, hshape).reshape(full_h))
        fim.append(plane(o + f_plane, fw, hc, hshape).reshape(full_h))
    return Masks(s, fre, fim)


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b))) / den
