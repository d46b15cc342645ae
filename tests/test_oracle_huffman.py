"""Pins of the oracle's entropy-coding stage (Sec. 4.1: the codes go through
a Huffman coding stage; Algorithm 1's Huffman step; Sec. 5 rebuilds the code
to decode), CPU only:

- canonical codewords reproduce the worked example printed in RFC 1951,
  Sec. 3.2.2 (lengths 3,3,3,3,3,2,4,4 for A..H);
- with a limit that does not bind, the code lengths cost exactly what the
  textbook Huffman construction (two lightest subtrees merged, written here
  with heapq) costs, and the code is complete (Kraft sum 1);
- with a binding limit, the cost equals the optimum found by brute force over
  every admissible length vector on tiny alphabets, and no length exceeds it;
- the bitstream decodes back to the codes, bit positions included.
"""
import heapq
import itertools

import numpy as np
import pytest

from oracle import oracle as O


def huffman_cost(counts):
    h = [int(c) for c in counts if c > 0]
    if len(h) <= 1:
        return sum(h)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def test_canonical_codes_rfc1951_example():
    ln = np.array([3, 3, 3, 3, 3, 2, 4, 4], dtype=np.uint8)
    code = O.huff_canonical(ln, 15)
    want = ["010", "011", "100", "101", "110", "00", "1110", "1111"]
    got = [format(int(c), f"0{int(l)}b") for c, l in zip(code, ln)]
    assert got == want


@pytest.mark.parametrize("seed", range(6))
def test_lengths_cost_equals_huffman_when_limit_is_loose(seed):
    rng = np.random.default_rng(seed)
    nsym = [2, 3, 17, 300, 4000, 65536][seed]
    hist = np.zeros(nsym, dtype=np.uint64)
    used = rng.choice(nsym, size=min(nsym, 2 + seed * 700), replace=False)
    hist[used] = (rng.pareto(1.2, used.size) * 50 + 1).astype(np.uint64)
    ln = O.huff_lengths(hist, 32)
    assert np.all((ln > 0) == (hist > 0))
    assert int((hist * ln).sum()) == huffman_cost(hist)
    kraft = sum(2.0 ** -int(v) for v in ln[ln > 0])
    assert kraft == pytest.approx(1.0, abs=1e-12)


def test_lengths_optimal_under_a_binding_limit():
    rng = np.random.default_rng(9)
    for trial in range(40):
        n = int(rng.integers(2, 7))
        lmax = int(rng.integers(max(1, int(np.ceil(np.log2(n)))), 5))
        if 2 ** lmax < n:
            continue
        w = np.concatenate([[1, 1, 2, 3, 5, 8, 13, 21][:n]]) if trial % 2 else \
            rng.integers(1, 1000, n)
        hist = np.asarray(w, dtype=np.uint64)
        ln = O.huff_lengths(hist, lmax)
        best = min(sum(int(a) * b for a, b in zip(hist, L))
                   for L in itertools.product(range(1, lmax + 1), repeat=n)
                   if sum(2.0 ** -b for b in L) <= 1.0)
        assert int((hist * ln).sum()) == best, (hist, lmax, ln)
        assert ln.max() <= lmax


def test_single_and_no_symbol():
    assert list(O.huff_lengths(np.array([0, 7, 0], dtype=np.uint64))) == [0, 1, 0]
    assert list(O.huff_lengths(np.zeros(4, dtype=np.uint64))) == [0, 0, 0, 0]


def test_bitstream_round_trip_and_positions():
    rng = np.random.default_rng(3)
    codes = np.clip(np.round(rng.laplace(32768, 40, 20000)), 1, 65535).astype(np.uint16)
    codes[::97] = 0
    hist = np.bincount(codes, minlength=65536).astype(np.uint64)
    ln = O.huff_lengths(hist)
    words, nbits = O.huff_encode(codes, ln)
    assert nbits == int((hist * ln).sum())
    back, end = O.huff_decode(words, codes.size, ln)
    assert end == nbits and np.array_equal(back, codes)
    # decoding from the middle: a block starting at its own bit offset
    off = int(ln[codes[:5000]].astype(np.int64).sum())
    part, end2 = O.huff_decode(words, 3000, ln, start=off)
    assert np.array_equal(part, codes[5000:8000])
    assert end2 == off + int(ln[codes[5000:8000]].astype(np.int64).sum())
    # the first codeword sits in the top bits of word 0
    cw = O.huff_canonical(ln)
    l0 = int(ln[codes[0]])
    assert int(words[0]) >> (32 - l0) == int(cw[codes[0]])
