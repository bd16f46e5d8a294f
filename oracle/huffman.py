"""CPU oracle of the lossless coding of the edits (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

What is computed (Alg. 1, LosslesslyCompressEdits; Sec. IV-B "Compaction,
quantization, and lossless compression of edits"; Sec. IV-D): the symbols of an
edit stream (the bytes of the flags, or the quantisation codes) are counted into
a global frequency table and Huffman-coded (Huffman 1952).  The paper follows the
Huffman stage with ZSTD, a third-party general-purpose compressor; that stage is
not part of this build.

Readings taken where the paper is silent
----------------------------------------
* Alphabet: the integers from the smallest to the largest symbol present.
* Tree: repeatedly merge the two lightest nodes; ties go to the node created
  first (leaves are created in symbol order, then each merged node in turn), so
  the tree -- and with it every code length -- is a function of the frequency
  table alone.  A single distinct symbol gets length 1.
* Length limit 32: while the longest code exceeds 32 bits, every non-zero count
  becomes ``(count + 1) // 2`` and the tree is rebuilt (the counts stay non-zero).
* Canonical codes: symbols sorted by (length, value); the first gets code 0, each
  next code is the previous plus one, shifted left by the increase in length.
* Bit order: codes are written most significant bit first into a stream of
  32-bit words, each word filled from its most significant bit down; the last
  word is padded with zeros.
* Chunk offsets: the bit position where symbol ``j * chunk`` starts, for every
  chunk (``chunk = 256``), so that a decoder can start at any chunk.
"""

from __future__ import annotations

import dataclasses
import heapq

import numpy as np

MAX_LEN = 32
CHUNK = 256


def histogram(sym: np.ndarray):
    """``(lo, counts)``: the global frequency table over the alphabet ``lo .. lo + len - 1``."""
    s = np.asarray(sym).astype(np.int64).ravel()
    if s.size == 0:
        return 0, np.zeros(0, dtype=np.int64)
    lo = int(s.min())
    return lo, np.bincount(s - lo).astype(np.int64)


def code_lengths(counts: np.ndarray) -> np.ndarray:
    """Huffman code length of every symbol (0 for an absent one), with the tie rule and the
    length limit of the module docstring."""
    c = np.asarray(counts, dtype=np.int64).copy()
    while True:
        lengths = _tree_lengths(c)
        if lengths.size == 0 or lengths.max() <= MAX_LEN:
            return lengths
        c = np.where(c > 0, (c + 1) // 2, 0)


def _tree_lengths(c: np.ndarray) -> np.ndarray:
    present = np.nonzero(c)[0]
    lengths = np.zeros(c.size, dtype=np.int64)
    if present.size == 0:
        return lengths
    if present.size == 1:
        lengths[present[0]] = 1
        return lengths
    # node ids: leaves 0 .. n-1 (symbol order), merged nodes n, n+1, ...
    heap = [(int(c[s]), i) for i, s in enumerate(present)]
    heapq.heapify(heap)
    parent = {}
    nid = present.size
    while len(heap) > 1:
        w1, a = heapq.heappop(heap)
        w2, b = heapq.heappop(heap)
        parent[a] = nid
        parent[b] = nid
        heapq.heappush(heap, (w1 + w2, nid))
        nid += 1
    root = heap[0][1]
    depth = {root: 0}
    for node in range(nid - 1, -1, -1):   # parents have larger ids than their children
        if node != root:
            depth[node] = depth[parent[node]] + 1
    for i, s in enumerate(present):
        lengths[s] = depth[i]
    return lengths


def canonical_codes(lengths: np.ndarray) -> np.ndarray:
    """Canonical code of every symbol (value of its ``length`` bits)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    codes = np.zeros(lengths.size, dtype=np.int64)
    order = sorted((int(l), s) for s, l in enumerate(lengths) if l > 0)
    code, prev = 0, None
    for l, s in order:
        if prev is not None:
            code = (code + 1) << (l - prev)
        else:
            code = 0
        codes[s] = code
        prev = l
    return codes


@dataclasses.dataclass
class Stream:
    lo: int
    lengths: np.ndarray      # per alphabet entry
    nbits: int
    words: np.ndarray        # uint32, ceil(nbits / 32)
    chunk_bits: np.ndarray   # int64, bit offset of symbol j * CHUNK


def encode(sym: np.ndarray) -> Stream:
    s = np.asarray(sym).astype(np.int64).ravel()
    lo, counts = histogram(s)
    lengths = code_lengths(counts)
    codes = canonical_codes(lengths)
    idx = s - lo
    L = lengths[idx]
    C = codes[idx]
    starts = np.concatenate([[0], np.cumsum(L)[:-1]]) if s.size else np.zeros(0, dtype=np.int64)
    nbits = int(L.sum())
    nwords = (nbits + 31) // 32
    bits = np.zeros(nwords * 32, dtype=np.uint8)
    for k in range(int(lengths.max()) if lengths.size else 0):
        # bit k of every code, counted from its most significant bit
        m = L > k
        bits[starts[m] + k] = (C[m] >> (L[m] - 1 - k)) & 1
    words = np.packbits(bits, bitorder="big").view(">u4").astype(np.uint32) if nwords else np.zeros(0, np.uint32)
    chunk_bits = starts[::CHUNK].astype(np.int64) if s.size else np.zeros(0, dtype=np.int64)
    return Stream(lo=lo, lengths=lengths, nbits=nbits, words=words, chunk_bits=chunk_bits)


def decode(st: Stream, n: int) -> np.ndarray:
    """Walk the stream bit by bit against the canonical code table (reference decoder)."""
    codes = canonical_codes(st.lengths)
    table = {(int(l), int(c)): st.lo + s for s, (l, c) in enumerate(zip(st.lengths, codes)) if l > 0}
    bits = np.unpackbits(np.asarray(st.words, dtype=">u4").view(np.uint8), bitorder="big")
    out = np.empty(n, dtype=np.int64)
    pos = 0
    for i in range(n):
        code, l = 0, 0
        while (l, code) not in table:
            code = (code << 1) | int(bits[pos])
            pos += 1
            l += 1
            if l > MAX_LEN:
                raise ValueError("invalid stream")
        out[i] = table[(l, code)]
    return out
