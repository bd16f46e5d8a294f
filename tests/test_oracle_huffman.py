"""Pins of the Huffman oracle (LosslesslyCompressEdits, Alg. 1; Sec. IV-B, IV-D):

- a hand-worked four-symbol table (lengths 1, 2, 3, 3; canonical codes 0, 10, 110, 111);
- the Huffman cost equals the sum of the weights of all merges, computed here with a plain
  sorted list (a property of the optimal prefix code), and lies in [H, H + 1) bits per symbol;
- Kraft equality, prefix freedom, canonical order;
- the length limit on Fibonacci counts (unlimited lengths would reach 44);
- round trips through the reference decoder and the chunk offsets.
"""

import math

import numpy as np
import pytest

from oracle import huffman as HF


def test_hand_worked_table():
    counts = np.array([5, 2, 1, 1])
    L = HF.code_lengths(counts)
    assert list(L) == [1, 2, 3, 3]
    C = HF.canonical_codes(L)
    assert [format(int(c), f"0{int(l)}b") for c, l in zip(C, L)] == ["0", "10", "110", "111"]
    # a stream with exactly these counts: 0 0 0 0 0 10 10 110 111 (15 bits, MSB first)
    st = HF.encode(np.array([0, 0, 0, 0, 0, 1, 1, 2, 3]))
    assert st.nbits == 15
    assert int(st.words[0]) == int("000001010110111" + "0" * 17, 2)
    # four symbols of one count each: a full tree of depth 2, codes 00 01 10 11
    st = HF.encode(np.array([0, 1, 2, 3]))
    assert list(st.lengths) == [2, 2, 2, 2] and int(st.words[0]) == int("00011011" + "0" * 24, 2)


def _merge_cost(counts):
    w = sorted(int(c) for c in counts if c > 0)
    if len(w) <= 1:
        return sum(w)  # one symbol: one bit each
    cost = 0
    while len(w) > 1:
        a, b = w[0], w[1]
        w = sorted(w[2:] + [a + b])
        cost += a + b
    return cost


@pytest.mark.parametrize("seed", range(8))
def test_huffman_cost_is_the_sum_of_merge_weights(seed):
    g = np.random.default_rng(seed)
    k = int(g.integers(2, 60))
    counts = g.integers(0, 1000, k)
    counts[g.integers(0, k)] += 1
    if np.count_nonzero(counts) < 2:
        counts[0] += 3
        counts[-1] += 2
    L = HF.code_lengths(counts)
    assert int(np.sum(L * counts)) == _merge_cost(counts)
    p = counts[counts > 0] / counts.sum()
    H = float(-np.sum(p * np.log2(p)))
    avg = float(np.sum(L * counts)) / counts.sum()
    assert H - 1e-12 <= avg < H + 1
    nz = L[counts > 0]
    assert sum(2.0 ** -int(l) for l in nz) == pytest.approx(1.0, abs=1e-12)   # Kraft equality
    assert np.all(L[counts == 0] == 0)


def test_canonical_codes_are_prefix_free_and_ordered():
    g = np.random.default_rng(9)
    counts = g.integers(1, 500, 40)
    L = HF.code_lengths(counts)
    C = HF.canonical_codes(L)
    words = [format(int(c), f"0{int(l)}b") for c, l in zip(C, L)]
    for i, a in enumerate(words):
        for j, b in enumerate(words):
            if i != j:
                assert not b.startswith(a)
    order = sorted(range(len(L)), key=lambda s: (int(L[s]), s))
    vals = [int(C[s]) << (32 - int(L[s])) for s in order]
    assert vals == sorted(vals) and len(set(vals)) == len(vals)


def test_length_limit():
    fib = [1, 1]
    while len(fib) < 46:
        fib.append(fib[-1] + fib[-2])
    counts = np.array(fib, dtype=np.int64)
    assert HF._tree_lengths(counts).max() > 32
    L = HF.code_lengths(counts)
    assert L.max() <= 32 and np.all(L > 0)
    assert sum(2.0 ** -int(l) for l in L) == pytest.approx(1.0, abs=1e-12)
    g = np.random.default_rng(10)
    sym = g.choice(len(fib), size=3000, p=counts / counts.sum())
    sym[:len(fib)] = np.arange(len(fib))   # every symbol present
    st = HF.encode(sym)
    np.testing.assert_array_equal(HF.decode(st, sym.size), sym)


@pytest.mark.parametrize("case", ["bytes", "codes", "single", "two", "empty", "wide"])
def test_round_trip_and_chunk_offsets(case):
    g = np.random.default_rng(11)
    if case == "bytes":
        sym = (g.random(20000) < 0.05).astype(np.int64) * g.integers(1, 256, 20000)
    elif case == "codes":
        sym = np.rint(g.standard_normal(9000) * 300).astype(np.int64)
    elif case == "single":
        sym = np.full(5000, -7)
    elif case == "two":
        sym = g.integers(0, 2, 10000) * 1000 - 500
    elif case == "empty":
        sym = np.zeros(0, dtype=np.int64)
    else:
        sym = g.integers(-(2 ** 20), 2 ** 20, 5000)
    st = HF.encode(sym)
    np.testing.assert_array_equal(HF.decode(st, sym.size), sym)
    assert st.words.size == (st.nbits + 31) // 32
    if sym.size:
        lo, counts = HF.histogram(sym)
        L = st.lengths[sym - lo]
        cs = np.concatenate([[0], np.cumsum(L)])
        np.testing.assert_array_equal(st.chunk_bits, cs[: sym.size][:: HF.CHUNK])
        assert st.nbits == int(cs[-1])
