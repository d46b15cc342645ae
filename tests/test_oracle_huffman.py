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

The codebook of the training phase (Sec. 4.3: one table from validation code
frequencies, reused for every block), with its escape for codes the
validation never produced:

- a worked example derived by hand (weights 3, 1 and an escape of weight 1:
  lengths 1, 2, 2; the stream of three codes written out bit by bit);
- the escape weighs the number of codes seen exactly once (a case where a
  weight of 1 would give another escape length) and sits last among the
  codewords of its length;
- with an escape the lengths stop at 16 bits (a case where the unlimited code
  goes beyond), without one (every code seen) they equal the 32-bit limited
  code of the counts; the code stays complete (Kraft sum 1);
- costs equal the textbook Huffman construction of the augmented weights
  when the limit does not bind;
- escaped and coded codes decode back, bit counts and positions included;
- the table's validation blocks (the compression simulated on a uniform
  sample of whole blocks): their code counts equal the counts recomputed
  here block by block, with splitmix64 written out from its published
  definition; every block at frac 1, none at frac 0, and about frac of them
  otherwise.
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


# --- the trained codebook (Sec. 4.3) ----------------------------------------------------------

def _hist(d):
    h = np.zeros(65536, dtype=np.uint64)
    for s, c in d.items():
        h[s] = c
    return h


def _bits(words, nbits):
    return "".join(format(int(w), "032b") for w in words)[:nbits]


def test_trained_codebook_worked_example():
    # weights: code 5 -> 3, code 7 -> 1, escape -> 1 (one code seen once).
    # Huffman: merge 7 and the escape (2), then with 5: lengths 1, 2, 2.
    # Canonical: 5 -> "0"; 7 -> "10", escape -> "11" (last of length 2).
    ln, esc = O.huff_trained_lengths(_hist({5: 3, 7: 1}))
    assert esc == 2 and ln[5] == 1 and ln[7] == 2 and ln[O.ESC] == 2
    assert int((ln > 0).sum()) == 3
    words, nbits = O.huff_encode_esc(np.array([5, 7, 9], dtype=np.uint16), ln)
    # "0" + "10" + "11" + the 16 bits of 9
    assert nbits == 21
    assert _bits(words, nbits) == "0" + "10" + "11" + "0000000000001001"
    assert int(words[0]) == 0x58004800
    back, end = O.huff_decode_esc(words, 3, ln)
    assert end == 21 and list(back) == [5, 7, 9]
    count, syms = O.huff_book(ln)
    assert list(count[:3]) == [0, 1, 2] and list(syms) == [5, 7, 0]


def test_escape_weight_is_the_singleton_count():
    # counts 100, 1, 1, 1: three codes seen once -> escape weight 3.
    # weights 100, 1, 1, 1, 3: merges 1+1, 1+2, 3+3, 6+100, so the escape
    # gets 2 bits.  A weight of 1 instead would make four equal leaves of
    # 3 bits under the heavy symbol.
    ln, esc = O.huff_trained_lengths(_hist({1: 100, 2: 1, 3: 1, 4: 1}))
    assert esc == 2
    assert [int(ln[s]) for s in (1, 2, 3, 4)] == [1, 4, 4, 3]
    # no code seen once: weight 1
    ln, esc = O.huff_trained_lengths(_hist({1: 10, 2: 4, 3: 4}))
    w = [10, 4, 4, 1]
    assert int(sum(a * b for a, b in zip(w, [ln[1], ln[2], ln[3], ln[O.ESC]]))) == \
        huffman_cost(w)
    assert esc == 3


@pytest.mark.parametrize("seed", range(4))
def test_trained_cost_equals_textbook_huffman_of_augmented_weights(seed):
    rng = np.random.default_rng(50 + seed)
    used = rng.choice(65536, size=[3, 40, 900, 3000][seed], replace=False)
    h = np.zeros(65536, dtype=np.uint64)
    h[used] = (rng.pareto(2.5, used.size) * 30 + 1).astype(np.uint64)
    ln, esc = O.huff_trained_lengths(h)
    ones = int((h == 1).sum())
    wesc = max(1, ones)
    # the 16-bit limit does not bind on these counts
    assert O.huff_lengths(np.append(h, np.uint64(wesc)), 62).max() <= 16
    assert ln.max() <= 16
    cost = int((h * ln[:65536]).sum()) + wesc * esc
    assert cost == huffman_cost(list(h[h > 0]) + [wesc])
    kraft = sum(2.0 ** -int(v) for v in ln[ln > 0])
    assert kraft == pytest.approx(1.0, abs=1e-12)
    # the escape is the last codeword of its length
    count, syms = O.huff_book(ln)
    first = int(count[:esc].sum())
    assert syms[first + int(count[esc]) - 1] == 0
    assert int((ln[:65536] == esc).sum()) == int(count[esc]) - 1


def test_trained_lengths_stop_at_16_bits_with_an_escape():
    # counts 2, 4, ..., 2^25 and the escape's 1: the unlimited code is 25 deep
    h = _hist({100 + i: 2 ** i for i in range(1, 26)})
    free = O.huff_lengths(np.append(h, np.uint64(1)), 62)
    assert free.max() == 25
    ln, esc = O.huff_trained_lengths(h)
    assert 0 < esc <= 16 and ln.max() == 16
    kraft = sum(2.0 ** -int(v) for v in ln[ln > 0])
    assert kraft == pytest.approx(1.0, abs=1e-12)


def test_every_code_seen_means_no_escape():
    rng = np.random.default_rng(8)
    h = (rng.pareto(1.1, 65536) * 3 + 1).astype(np.uint64)
    ln, esc = O.huff_trained_lengths(h)
    assert esc == 0 and ln[O.ESC] == 0
    assert np.array_equal(ln[:65536], O.huff_lengths(h, 32))


def test_empty_validation_escapes_everything():
    ln, esc = O.huff_trained_lengths(np.zeros(65536, dtype=np.uint64))
    assert esc == 1 and int((ln > 0).sum()) == 1
    words, nbits = O.huff_encode_esc(np.array([3, 65535], dtype=np.uint16), ln)
    assert nbits == 34
    assert _bits(words, nbits) == "0" + format(3, "016b") + "0" + format(65535, "016b")


def test_trained_stream_round_trip_with_escapes():
    rng = np.random.default_rng(12)
    val = np.clip(np.round(rng.laplace(32768, 30, 30000)), 1, 65535).astype(np.uint16)
    ln, esc = O.huff_trained_lengths(np.bincount(val, minlength=65536).astype(np.uint64))
    assert esc > 0
    codes = np.clip(np.round(rng.laplace(32768, 60, 20000)), 0, 65535).astype(np.uint16)
    codes[::101] = 0
    per = np.array([int(ln[c]) if ln[c] else esc + 16 for c in codes])
    assert (ln[codes] == 0).sum() > 100  # escapes happen
    words, nbits = O.huff_encode_esc(codes, ln)
    assert nbits == int(per.sum())
    back, end = O.huff_decode_esc(words, codes.size, ln)
    assert end == nbits and np.array_equal(back, codes)
    off = int(per[:7000].sum())
    part, end2 = O.huff_decode_esc(words, 5000, ln, start=off)
    assert np.array_equal(part, codes[7000:12000])
    assert end2 == off + int(per[7000:12000].sum())


# --- the table's validation blocks -------------------------------------------------------------

def _splitmix64(state):
    m = (1 << 64) - 1
    z = (state + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def _blocks_in_stream_order(shape, B):
    nb = [-(-s // B) for s in shape]
    for bi in np.ndindex(*nb):
        yield int(np.prod([min(B, s - b * B) for s, b in zip(shape, bi)]))


@pytest.mark.parametrize("shape,B", [((37, 20, 19), 8), ((130, 71), 16), ((1001,), 64),
                                     ((9, 9, 9), 4)])
def test_table_hist_is_the_selected_blocks_codes(shape, B):
    rng = np.random.default_rng(len(shape) * 7 + B)
    n = int(np.prod(shape))
    codes = np.clip(np.round(rng.laplace(32768, 40, n)), 0, 65535).astype(np.uint16)
    seed, frac = 0x5EED + B, 0.3
    hist, nsel = O.table_hist(codes, shape, B, frac, seed)
    want = np.zeros(65536, dtype=np.uint64)
    pos = k = 0
    for b, size in enumerate(_blocks_in_stream_order(shape, B)):
        u = (_splitmix64(seed ^ b) >> 11) * 2.0 ** -53
        if u < frac:
            k += 1
            want += np.bincount(codes[pos:pos + size], minlength=65536).astype(np.uint64)
        pos += size
    assert pos == n and nsel == k and np.array_equal(hist, want)
    nblocks = sum(1 for _ in _blocks_in_stream_order(shape, B))
    assert abs(nsel - frac * nblocks) <= 4 * np.sqrt(frac * (1 - frac) * nblocks) + 1
    full, nall = O.table_hist(codes, shape, B, 1.0, seed)
    assert nall == nblocks
    assert np.array_equal(full, np.bincount(codes, minlength=65536).astype(np.uint64))
    none, nz = O.table_hist(codes, shape, B, 0.0, seed)
    assert nz == 0 and not none.any()
