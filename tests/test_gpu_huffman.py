"""Huffman coding of the edit streams on the GPU (LosslesslyCompressEdits, Alg. 1; Sec. IV-B,
IV-D) against the oracle, through the C ABI: the code lengths, the 32-bit words, the bit count
and the chunk offsets are bit-exact (the tree's tie rule and the length limit are the same on
both sides), and decoding returns the symbols.  Streams: the flag bytes and codes of an
encoded field, synthetic byte and code streams, a single symbol, the length limit, empty.
"""

import numpy as np
import pytest

from oracle import huffman as HF
from paper_2601_01596_amd import ffcz as F
from paper_2601_01596_amd import workloads as W
from tests.progress import say

pytestmark = pytest.mark.gpu

HDR = 64


def _parse(stream, width):
    """Split a device stream into (lengths, chunk offsets, words, header fields)."""
    b = stream.cpu().numpy()
    hd = b[:HDR].view(np.int64)
    magic_width = b[:8].view(np.uint32)
    assert int(magic_width[0]) == 0x46554846 and int(magic_width[1]) == width
    nsym, lo, nalpha, nbits, nch = (int(v) for v in hd[1:6])
    off_len = HDR
    off_ch = (off_len + nalpha + 15) // 16 * 16
    off_w = (off_ch + 8 * nch + 15) // 16 * 16
    lengths = b[off_len: off_len + nalpha].astype(np.int64)
    chunks = b[off_ch: off_ch + 8 * nch].view(np.uint64).astype(np.int64)
    words = b[off_w: off_w + 4 * ((nbits + 31) // 32)].view(np.uint32)
    return dict(nsym=nsym, lo=lo, nalpha=nalpha, nbits=nbits, lengths=lengths, chunks=chunks, words=words)


def _check(sym_np, dtype):
    import torch
    width = 1 if dtype == np.uint8 else 4
    t = torch.from_numpy(np.ascontiguousarray(sym_np.astype(dtype))).cuda()
    stream, sizes = F.huffman_compress(t)
    got = _parse(stream, width)
    ref = HF.encode(sym_np.astype(np.int64))
    assert got["nsym"] == sym_np.size
    if sym_np.size:
        assert got["lo"] == ref.lo and got["nalpha"] == ref.lengths.size
        np.testing.assert_array_equal(got["lengths"], ref.lengths)
        assert got["nbits"] == ref.nbits
        np.testing.assert_array_equal(got["chunks"], ref.chunk_bits)
        np.testing.assert_array_equal(got["words"], ref.words)
    back = F.huffman_decompress(stream, sym_np.size, t.dtype, int(sizes.nalpha))
    np.testing.assert_array_equal(back.cpu().numpy()[: sym_np.size], sym_np.astype(dtype))
    return got


@pytest.mark.parametrize("case", ["bytes", "codes", "single", "two", "wide", "empty", "one", "ragged"])
def test_streams_match_the_oracle_bit_for_bit(case):
    g = np.random.default_rng(3)
    if case == "bytes":
        sym, dt = ((g.random(300000) < 0.04) * g.integers(1, 256, 300000)).astype(np.int64), np.uint8
    elif case == "codes":
        sym, dt = np.rint(g.standard_normal(200000) * 900).astype(np.int64), np.int32
    elif case == "single":
        sym, dt = np.full(70000, -12345), np.int32
    elif case == "two":
        sym, dt = g.integers(0, 2, 100000) * 255, np.uint8
    elif case == "wide":
        sym, dt = g.integers(-(2 ** 20), 2 ** 20, 50000), np.int32
    elif case == "empty":
        sym, dt = np.zeros(0, np.int64), np.int32
    elif case == "one":
        sym, dt = np.array([7]), np.uint8
    else:  # a length that fills no word or chunk exactly
        sym, dt = np.rint(g.laplace(0, 30, 1024 * 7 + 333)).astype(np.int64), np.int32
    _check(sym, dt)


def test_length_limit_matches_the_oracle():
    fib = [1, 1]
    while len(fib) < 46:
        fib.append(fib[-1] + fib[-2])
    p = np.array(fib, dtype=np.float64)
    g = np.random.default_rng(4)
    sym = g.choice(len(fib), size=200000, p=p / p.sum())
    sym[: len(fib)] = np.arange(len(fib))
    got = _check(sym, np.int32)
    assert got["lengths"].max() <= 32


def test_edit_streams_of_an_encoded_field():
    import torch
    prob = W.config_lognormal(64, np.float32)
    enc = F.encode(torch.from_numpy(prob.x).cuda(), torch.from_numpy(prob.xb).cuda(), prob.E, prob.Delta,
                   prob.max_iter)
    assert enc.status == F.OK
    total_in = total_out = 0
    for name, t in (("spatial flags", enc.spat_flags), ("spatial codes", enc.spat_codes),
                    ("frequency flags", enc.freq_flags), ("frequency codes", enc.freq_codes)):
        sym = t.cpu().numpy().astype(np.int64)
        got = _check(sym, np.uint8 if t.dtype == torch.uint8 else np.int32)
        nb = (got["nbits"] + 7) // 8
        total_in += t.numel() * t.element_size()
        total_out += nb
        say(f"[huffman] {name}: {t.numel()} symbols, {t.numel() * t.element_size()} -> {nb} bytes")
    say(f"[huffman] edits of the 64^3 field: {total_in} -> {total_out} bytes")
    assert total_out < total_in


def test_corrupt_streams_are_refused():
    # the decoder checks the header (magic, width, chunk count) and the stored code lengths
    # (at most 32 bits, Kraft sum at most 1) before it launches; a corrupt stream is refused
    import torch
    g = np.random.default_rng(5)
    sym = np.rint(g.standard_normal(5000) * 40).astype(np.int32)
    stream, sizes = F.huffman_compress(torch.from_numpy(sym).cuda())
    n, na = sym.size, int(sizes.nalpha)
    good = F.huffman_decompress(stream, n, torch.int32, na)
    np.testing.assert_array_equal(good.cpu().numpy()[:n], sym)

    def refused(mutate):
        b = stream.clone()
        mutate(b)
        with pytest.raises(F.FFCzError) as ei:
            F.huffman_decompress(b, n, torch.int32, na)
        assert ei.value.status == F.E_INVALID

    def bad_magic(b):
        b[0] ^= 0xFF

    def bad_chunks(b):  # header word 5 (int64): the chunk count
        h = b[:HDR].cpu().numpy().view(np.int64).copy()
        h[5] += 1
        b[:HDR] = torch.from_numpy(h.view(np.uint8)).cuda()

    def over_kraft(b):  # every present symbol gets a 1-bit code
        lens = b[HDR:HDR + na]
        b[HDR:HDR + na] = torch.where(lens > 0, torch.ones_like(lens), lens)

    def too_long(b):
        i = int(np.argmax(b[HDR:HDR + na].cpu().numpy()))
        b[HDR + i] = 33

    for m in (bad_magic, bad_chunks, over_kraft, too_long):
        refused(m)
    with pytest.raises(F.FFCzError):  # wrong symbol width
        F.huffman_decompress(stream, n, torch.uint8, na)

