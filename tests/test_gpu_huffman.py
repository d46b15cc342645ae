"""GPU parity of the Huffman stage (Sec. 4.1 coding stage; Algorithm 1's
Huffman step; Sec. 5 decoding).

For each field the stream with Huffman-coded codes is checked against the
oracle: its bit section equals, word for word, the oracle's canonical
encoding of the oracle's codes under the stream's code lengths; those lengths
cost exactly the optimum of the oracle's package-merge (32-bit limit) on the
histogram of the oracle's codes; every block's bit size is the sum of its
codes' lengths; raw values are the oracle's; and the reconstruction equals
the oracle's bit for bit.  Several optimal codebooks can exist, so the
lengths themselves are checked for validity (Kraft, canonical order), not
for equality."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth
from tests.test_gpu_codec import _case, assert_bound, dev, random_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


def _block_sizes(codes, shape, B, ln):
    """Bits of every block (stream order) from the codes in stream order."""
    nb = [-(-s // B) for s in shape]
    sizes, pos = [], 0
    lens = ln[codes].astype(np.int64)
    for bi in np.ndindex(*nb):
        ext = [min(B, s - b * B) for s, b in zip(shape, bi)]
        n = int(np.prod(ext))
        sizes.append(int(lens[pos:pos + n].sum()))
        pos += n
    return np.array(sizes, dtype=np.int64)


def _check_huffman_stream(stream, codes_ref, shape, B):
    sec = pwrel.sections(stream)
    h = sec["header"]
    assert h["flags"] & pwrel.HF_HUFFMAN and h["off_codes"] == 0
    cnt = sec["huff_count"].cpu().numpy().view(np.uint32)
    syms = sec["huff_syms"].cpu().numpy().view(np.uint16)
    ln = pwrel.codebook_lengths(cnt, syms)
    hist = np.bincount(codes_ref, minlength=65536).astype(np.uint64)
    # a prefix code over exactly the used symbols, in canonical order
    assert np.array_equal(np.flatnonzero(ln), np.flatnonzero(hist))
    assert sum(int(cnt[l]) * 2.0 ** -l for l in range(1, 33)) <= 1.0
    keys = [(int(ln[s]), int(s)) for s in syms]
    assert keys == sorted(keys)
    # optimal: the oracle's package-merge cost under the same limit
    nbits = int((hist.astype(np.int64) * ln.astype(np.int64)).sum())
    assert h["n_bits"] == nbits == int(
        (hist.astype(np.int64) * O.huff_lengths(hist, 32).astype(np.int64)).sum())
    # the bits: the oracle's canonical encoding of the oracle's codes, word for word
    words_ref, nb_ref = O.huff_encode(codes_ref, ln, lmax=32)
    assert nb_ref == nbits
    bits = sec["bits"].cpu().numpy().view(np.uint32)
    assert np.array_equal(bits, words_ref[:bits.size])
    dec, end = O.huff_decode(bits, codes_ref.size, ln, lmax=32)
    assert end == nbits and np.array_equal(dec, codes_ref)
    sizes = sec["sizes"].cpu().numpy()
    sizes = sizes.view(np.uint16 if h["size_bytes"] == 2 else np.uint32).astype(np.int64)
    assert np.array_equal(sizes, _block_sizes(codes_ref, shape, B, ln))
    return sec


def _hcase(name):
    if name == "ones_single_symbol":   # every grid value 0: every code is 2^15, one symbol
        return np.ones((40, 40, 40), dtype=np.float32), 1e-2, 8, None, False
    if name == "zeros_two_symbols":
        return np.zeros((64, 64, 64), dtype=np.float32), 1e-2, 8, None, False
    return _case(name)


HUFF_CASES = ["ones_single_symbol", "zeros_two_symbols", "config0_bumps64", "grf_ragged_1e-3", "grf_ragged_indep", "grf_B4_H32",
              "grf_B16_H8", "zonal_2d", "grf_2d_B64", "grf_1d_halo", "f64_1e-4", "lorenzo_only",
              "single_point", "all_zero", "tiny_1d", "pencil_long"]


@pytest.mark.parametrize("name", HUFF_CASES)
def test_huffman_stream_vs_oracle(ctx, name):
    x, eps, B, model, indep = _hcase(name)
    print(f"[huffman] {name} {x.shape} B={B}", flush=True)
    use_net = model is not None
    mode = O.MODE_PLAIN if use_net else O.MODE_LORENZO
    ref = O.compress(x, eps, B, model, mode, independent=indep)
    stream = ctx.compress(dev(x), eps, B, model, use_net=use_net, independent=indep,
                          entropy=True)
    plain = ctx.compress(dev(x), eps, B, model, use_net=use_net, independent=indep)
    h = pwrel.header(stream)
    if not h["flags"] & pwrel.HF_HUFFMAN:
        # the codebook would cost more than it saves: the 16-bit stream, byte for byte
        assert name in ("grf_ragged_1e-3", "grf_ragged_indep", "f64_1e-4", "single_point",
                        "tiny_1d", "all_zero"), name
        assert np.array_equal(stream.cpu().numpy(), plain.cpu().numpy())
        return
    assert stream.numel() < plain.numel()
    sec = _check_huffman_stream(stream, ref["codes"], x.shape, B)
    assert np.array_equal(sec["counts"].cpu().numpy().view(np.uint32), ref["counts"])
    assert np.array_equal(sec["raw"].cpu().numpy().view(np.uint8), ref["raw"].view(np.uint8))
    xh = ctx.decompress(stream).cpu().numpy()
    ref_xh, _ = O.decompress(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, B, model,
                             mode, independent=indep)
    assert np.array_equal(xh.view(np.uint8), ref_xh.view(np.uint8))
    assert_bound(x, xh, eps)


@pytest.mark.parametrize("indep", [False, True])
def test_huffman_learned_judge_stream(ctx, indep):
    """BF16 network with the per-block judge: the Huffman stream holds the
    same codes as the 16-bit stream of the same call and decodes to the same
    field; the stored size matches the exact Huffman size of the histogram."""
    x = synth.lognormal_grf((40, 48, 72), seed=21, decades=8, neg_frac=0.1, zero_frac=0.005)
    xd = dev(x)
    model = random_model(3, 32, 21)
    model["precision"] = 1
    plain = ctx.compress(xd, 1e-2, 8, model, judge=True, independent=indep)
    huff = ctx.compress(xd, 1e-2, 8, model, judge=True, independent=indep, entropy=True)
    ps = pwrel.sections(plain)
    codes = ps["codes"].cpu().numpy().view(np.uint16)
    hs = _check_huffman_stream(huff, codes, x.shape, 8)
    assert np.array_equal(hs["bflags"].cpu().numpy(), ps["bflags"].cpu().numpy())
    hist = ctx.histogram(ps["codes"])
    assert hs["header"]["n_bits"] == pwrel.huffman_bits(hist)[0]
    a = ctx.decompress(plain).cpu().numpy()
    b = ctx.decompress(huff).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert_bound(x, b, 1e-2)


def test_huffman_corrupt_codebook_is_rejected(ctx):
    """Length counts that do not describe the stored symbols are found on the
    host before any decoding kernel runs."""
    x = synth.lognormal_grf((20, 20, 20), seed=3)
    s = ctx.compress(dev(x), 1e-2, 8, None, use_net=False, entropy=True).clone()
    h = pwrel.header(s)
    off = h["off_huff"] + 4 * 32          # count[32]
    s[off:off + 4] = torch.tensor([1, 0, 0, 0], dtype=torch.uint8, device=s.device)
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.decompress(s)
    assert e.value.status == pwrel.ECORRUPT
