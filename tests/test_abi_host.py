"""CPU-side checks of the HIP library's C ABI: the library loads, exports
every entry point include/pwrel.h declares, and its host-only logic
(argument checks, bounds, header validation, Huffman sizing, network
initialisation) behaves as documented.  No compute call is made here."""
import ctypes as C
import heapq
import os
import re
import struct

import numpy as np
import pytest

from oracle import oracle as O
from paper_2309_09778_amd import pwrel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pwrel.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pwrel_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pwrel.lib()
    decl = declared_symbols()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(pwrel.exported_symbols()) == decl


def test_nm_lists_symbols_as_extern_c():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", pwrel.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    names = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in declared_symbols():
        assert name in names, name


def test_argument_checks():
    assert pwrel.check_args((64, 64, 64), pwrel.F32, 1e-2, 8) == pwrel.OK
    bad = [((64, 64, 64), pwrel.F32, 0.0, 8), ((64, 64, 64), pwrel.F32, 1.0, 8),
           ((64, 64, 64), pwrel.F32, 1e-2, 17), ((64, 64, 64), pwrel.F32, 1e-2, 1),
           ((64, 0, 64), pwrel.F32, 1e-2, 8), ((64, 64), 7, 1e-2, 8),
           ((1800, 3600), pwrel.F32, 1e-2, 65), ((10,), pwrel.F64, 1e-18, 8)]
    for shape, dt, eps, b in bad:
        assert pwrel.check_args(shape, dt, eps, b) == pwrel.EINVAL, (shape, dt, eps, b)
    assert pwrel.check_args((4097,), pwrel.F64, 1e-3, 4096) == pwrel.OK


def test_compress_bound_covers_every_section():
    n = 512 ** 3
    nb = 64 ** 3
    b = pwrel.compress_bound((512, 512, 512), pwrel.F32, 8)
    # every section of a 16-bit-code stream, or of a Huffman stream: a codebook of at most
    # 65,536 symbols (33 length counts + 2 bytes a symbol), 4 bytes of bit size a block and
    # at most 16 bits a code
    huff = 4 * 33 + 2 * 65536 + 4 * nb
    assert b >= 512 + C.sizeof(pwrel.Mlp) + nb + 4 * nb + 2 * n + 4 * n + huff
    assert b < 512 + 4096 + nb + 4 * nb + 2 * n + 4 * n + huff
    assert pwrel.compress_bound((8, 8, 8), 3, 8) == 0


def _valid_header(n=(10, 12), block=4, flags=0, dtype=pwrel.F32, n_raw=3):
    h = pwrel.Header()
    h.magic, h.version, h.dtype, h.ndim = 0x4C455750, 1, dtype, len(n)
    for d, v in enumerate(n):
        h.dims[d] = v
    h.block, h.flags = block, flags
    h.eps, h.w, h.r, h.b_a = 1e-2, 0.0287, 34.8, 0.01435
    h.Lp, h.Ln, h.p_zero, h.b_sign, h.delta = 0.0, 2.0, -4389, 70, 0
    h.p_max = 141
    N = int(np.prod(n))
    nb = int(np.prod([-(-v // block) for v in n]))
    h.n, h.nblocks, h.n_raw = N, nb, n_raw
    al = lambda v: (v + 255) // 256 * 256
    o = 512
    h.off_model = o
    if flags & pwrel.HF_NET:
        o = al(o + C.sizeof(pwrel.Mlp))
    h.off_bflags = o
    if flags & pwrel.HF_JUDGE:
        o = al(o + nb)
    h.off_counts = o
    o = al(o + 4 * nb)
    h.off_codes = o
    o = al(o + 2 * N)
    h.off_raw = o
    h.total_size = o + n_raw * (4 if dtype == pwrel.F32 else 8)
    return h


def _bytes(h):
    return bytes(C.string_at(C.addressof(h), C.sizeof(h))) + b"\0" * (512 - C.sizeof(h))


def test_header_validation_accepts_consistent_and_rejects_corrupt():
    h = _valid_header()
    d = pwrel.read_header_bytes(_bytes(h), size=h.total_size)
    assert d["n"] == 120 and d["nblocks"] == 9
    for flags in (pwrel.HF_NET, pwrel.HF_NET | pwrel.HF_JUDGE, pwrel.HF_INDEPENDENT):
        hh = _valid_header(flags=flags)
        pwrel.read_header_bytes(_bytes(hh), size=hh.total_size)
    corruptions = [("magic", 0x12345678), ("version", 2), ("dtype", 5), ("ndim", 4),
                   ("n", 121), ("nblocks", 8), ("off_codes", 1024), ("n_raw", 4),
                   ("total_size", 10 ** 9), ("w", -1.0), ("eps", 2.0), ("status", -5),
                   ("delta", -1), ("flags", 64), ("p_max", 70)]
    for field, val in corruptions:
        hh = _valid_header()
        setattr(hh, field, val)
        with pytest.raises(pwrel.PwrelError) as e:
            pwrel.read_header_bytes(_bytes(hh), size=h.total_size)
        assert e.value.status == pwrel.ECORRUPT, field
    with pytest.raises(pwrel.PwrelError):   # truncated stream
        pwrel.read_header_bytes(_bytes(h), size=h.total_size - 1)


def _huffman_ref(counts):
    counts = [c for c in counts if c]
    if len(counts) == 1:
        return counts[0]
    heap = [(c, i) for i, c in enumerate(counts)]
    heapq.heapify(heap)
    total, nxt = 0, len(counts)
    while len(heap) > 1:
        a, _ = heapq.heappop(heap)
        b, _ = heapq.heappop(heap)
        total += a + b           # each merge adds one bit to every symbol below it
        heapq.heappush(heap, (a + b, nxt))
        nxt += 1
    return total


def test_huffman_bits_matches_textbook_merge_cost():
    rng = np.random.default_rng(1)
    for trial in range(20):
        hist = np.zeros(65536, dtype=np.uint64)
        k = rng.integers(1, 300)
        idx = rng.choice(65536, size=k, replace=False)
        hist[idx] = rng.integers(1, 10 ** 6, size=k)
        bits, maxlen = pwrel.huffman_bits(hist)
        assert bits == _huffman_ref(hist.tolist())
    # two equiprobable symbols: one bit each
    hist = np.zeros(65536, dtype=np.uint64)
    hist[5] = hist[9] = 1000
    assert pwrel.huffman_bits(hist) == (2000, 1)


def test_library_network_init_equals_oracle_init():
    for ndim, H in ((3, 16), (3, 32), (2, 8), (1, 2)):
        a = pwrel.mlp_init(ndim, H, 0.01, 7)
        b = O.mlp_init(ndim, H, 0.01, 7)
        for k in ("w1", "b1", "v"):
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (ndim, H, k)
        assert a["b2"] == b["b2"] and a["alpha"] == b["alpha"]


def test_create_without_gpu_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except Exception:
        pass
    with pytest.raises(pwrel.PwrelError):
        pwrel.Context(0)


def test_model_struct_fills_every_field():
    """The C struct built from a model dict by whole-array copies holds the
    same bytes as one filled field by field; a built struct passes through;
    networks beyond the struct's fixed sizes are refused."""
    rng = np.random.default_rng(5)
    for H, K in ((32, 6), (7, 2), (1, 0)):
        m = {"alpha": 0.03, "w1": rng.standard_normal((H, K)).astype(np.float32),
             "b1": rng.standard_normal(H).astype(np.float32),
             "v": rng.standard_normal(H).astype(np.float32), "b2": -0.25, "precision": 1}
        ref = pwrel.Mlp()
        ref.hidden, ref.inputs, ref.alpha = H, K, np.float32(0.03)
        for j in range(H):
            for k in range(K):
                ref.w1[j][k] = float(m["w1"][j, k])
            ref.b1[j] = float(m["b1"][j])
            ref.v[j] = float(m["v"][j])
        ref.b2, ref.precision = -0.25, 1
        s = pwrel.model_struct(m)
        assert bytes(s) == bytes(ref)
        assert pwrel.model_struct(s) is s
        back = pwrel.model_dict(s)
        for key in ("w1", "b1", "v"):
            assert np.array_equal(back[key], m[key])
    with pytest.raises(ValueError):
        pwrel.model_struct({"alpha": 0.0, "w1": np.zeros((33, 6), np.float32),
                            "b1": np.zeros(33, np.float32), "v": np.zeros(33, np.float32),
                            "b2": 0.0})


# --- trained network kept between fields (Sec. 5): save / load ---------------------------

def _trained_like(ndim, H, seed):
    rng = np.random.default_rng(seed)
    m = pwrel.mlp_init(ndim, H, 0.01, seed)
    K = (1 << ndim) - 2
    m["w1"] = (m["w1"] + rng.normal(0, 0.3, (H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 1, H).astype(np.float32)
    m["v"] = rng.normal(0, 1, H).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal()))
    m["precision"] = 1
    return m


@pytest.mark.parametrize("ndim,H", [(3, 32), (2, 16), (1, 4)])
def test_model_save_load_round_trip(ndim, H):
    m = _trained_like(ndim, H, ndim * 10 + H)
    data = pwrel.model_save(m)
    K = (1 << ndim) - 2
    assert len(data) == 24 + 4 * (H * K + 2 * H + 1) + 8
    assert data[:4] == b"PWMD" and struct.unpack("<I", data[4:8])[0] == 1
    back = pwrel.model_load(data)
    for k in ("w1", "b1", "v"):
        assert np.array_equal(np.asarray(back[k]).view(np.uint32),
                              np.asarray(m[k], np.float32).view(np.uint32)), k
    assert np.float32(back["b2"]) == np.float32(m["b2"])
    assert back["precision"] == 1 and back["alpha"] == np.float32(0.01)
    # the bytes are a fixed function of the network
    assert pwrel.model_save(back) == data


def test_model_load_rejects_damage():
    data = pwrel.model_save(_trained_like(3, 16, 5))
    for i in (0, 5, 9, 30, len(data) - 20, len(data) - 1):
        bad = bytearray(data)
        bad[i] ^= 0x10
        with pytest.raises(pwrel.PwrelError) as e:
            pwrel.model_load(bytes(bad))
        assert e.value.status == pwrel.ECORRUPT, i
    for cut in (0, 10, len(data) - 1):
        with pytest.raises(pwrel.PwrelError) as e:
            pwrel.model_load(data[:cut])
        assert e.value.status == pwrel.ECORRUPT
    with pytest.raises(pwrel.PwrelError) as e:
        pwrel.model_load(data + b"\0")
    assert e.value.status == pwrel.ECORRUPT


def test_model_save_capacity_and_invalid_network():
    L = pwrel.lib()
    m = pwrel.model_struct(_trained_like(3, 8, 1))
    size = C.c_uint64(0)
    assert L.pwrel_model_save(C.byref(m), None, 0, C.byref(size)) == pwrel.ENOSPC
    need = size.value
    buf = C.create_string_buffer(need)
    assert L.pwrel_model_save(C.byref(m), C.cast(buf, C.c_void_p), need - 1,
                              C.byref(size)) == pwrel.ENOSPC
    assert L.pwrel_model_save(C.byref(m), C.cast(buf, C.c_void_p), need, C.byref(size)) == 0
    m.hidden = 40
    assert L.pwrel_model_save(C.byref(m), C.cast(buf, C.c_void_p), need,
                              C.byref(size)) == pwrel.EINVAL
    m.hidden = 8
    m.w1[0][0] = float("nan")
    assert L.pwrel_model_save(C.byref(m), C.cast(buf, C.c_void_p), need,
                              C.byref(size)) == pwrel.EINVAL


def _oracle_cost(hist, lmax):
    ln = O.huff_lengths(hist, lmax)
    return int((hist.astype(np.int64) * ln.astype(np.int64)).sum())


@pytest.mark.parametrize("kind", ["uniform", "zipf", "geometric", "one", "two", "wide"])
def test_library_codebook_is_optimal_and_canonical(kind):
    """The stream's codebook (library host code) costs exactly the optimum
    that the oracle's package-merge reaches with the same 32-bit limit, its
    lengths satisfy Kraft, and its symbols are in canonical order."""
    rng = np.random.default_rng(hash(kind) % 1000)
    hist = np.zeros(65536, dtype=np.uint64)
    if kind == "uniform":
        idx = rng.choice(65536, 500, replace=False)
        hist[idx] = rng.integers(1, 1000, 500)
    elif kind == "zipf":
        idx = rng.choice(65536, 3000, replace=False)
        hist[idx] = (1e7 / np.arange(1, 3001) ** 1.3).astype(np.uint64) + 1
    elif kind == "geometric":   # deep tree (lengths in the twenties)
        idx = 32768 + np.arange(-30, 31)
        hist[idx] = (2.0 ** (30 - np.abs(np.arange(-30, 31)))).astype(np.uint64)
    elif kind == "one":
        hist[32768] = 12345
    elif kind == "two":
        hist[0], hist[65535] = 3, 7
    else:
        hist[:] = rng.integers(0, 50, 65536)
    cnt, syms, nbits = pwrel.huffman_codebook(hist)
    used = np.flatnonzero(hist)
    assert cnt[0] == 0 and int(cnt.sum()) == used.size == syms.size
    ln = pwrel.codebook_lengths(cnt, syms)
    assert np.array_equal(np.flatnonzero(ln), used)
    assert sum(int(cnt[l]) * 2.0 ** -l for l in range(1, 33)) <= 1.0
    assert int((hist.astype(np.int64) * ln.astype(np.int64)).sum()) == nbits
    keys = [(int(ln[s]), int(s)) for s in syms]
    assert keys == sorted(keys)
    assert nbits == _oracle_cost(hist, 32)
    if used.size > 1:
        assert nbits == pwrel.huffman_bits(hist)[0]   # the 32-bit limit did not bind


def test_library_codebook_caps_lengths_at_32_bits():
    """Fibonacci counts make the optimal unlimited code 39 bits deep; the
    stream's codebook caps every length at 32 and stays a prefix code, at a
    cost no lower than the limited optimum of the oracle."""
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    hist = np.zeros(65536, dtype=np.uint64)
    hist[100:140] = fib
    assert pwrel.huffman_bits(hist)[1] == 39
    cnt, syms, nbits = pwrel.huffman_codebook(hist)
    ln = pwrel.codebook_lengths(cnt, syms)
    assert ln.max() <= 32 and sum(int(cnt[l]) * 2.0 ** -l for l in range(1, 33)) <= 1.0
    assert nbits >= _oracle_cost(hist, 32)
    assert nbits == int((hist.astype(np.int64) * ln.astype(np.int64)).sum())


def test_huffman_header_validation():
    """A Huffman stream's header: sections after the counts in the stated order,
    256-byte aligned; inconsistent offsets, sizes or symbol counts are corrupt."""
    n, block, nraw, nsym, nbits = (10, 12), 4, 3, 7, 333
    h = _valid_header(n=n, block=block, n_raw=nraw)
    al = lambda v: (v + 255) // 256 * 256
    nb = h.nblocks
    h.flags = pwrel.HF_HUFFMAN
    h.off_huff = h.off_codes
    h.off_codes = 0
    h.n_sym, h.n_bits, h.size_bytes = nsym, nbits, 2
    h.off_sizes = al(h.off_huff + 4 * 33 + 2 * nsym)
    h.off_bits = al(h.off_sizes + 2 * nb)
    h.off_raw = al(h.off_bits + 4 * ((nbits + 31) // 32))
    h.total_size = h.off_raw + 4 * nraw
    d = pwrel.read_header_bytes(_bytes(h), size=h.total_size)
    assert d["n_sym"] == nsym and d["off_bits"] == h.off_bits
    for field, val in [("off_codes", 512), ("off_sizes", h.off_sizes + 256), ("n_sym", 0),
                       ("size_bytes", 4), ("n_bits", 16 * 120 + 1), ("off_raw", h.off_raw + 256),
                       ("off_huff", h.off_huff + 256)]:
        hh = pwrel.Header.from_buffer_copy(bytes(h))
        setattr(hh, field, val)
        with pytest.raises(pwrel.PwrelError) as e:
            pwrel.read_header_bytes(_bytes(hh), size=h.total_size + 4096)
        assert e.value.status == pwrel.ECORRUPT, field
    # an escape of up to 16 bits is valid, a longer one corrupt
    hh = pwrel.Header.from_buffer_copy(bytes(h))
    hh.esc_len = 16
    assert pwrel.read_header_bytes(_bytes(hh), size=h.total_size)["esc_len"] == 16
    hh.esc_len = 17
    with pytest.raises(pwrel.PwrelError):
        pwrel.read_header_bytes(_bytes(hh), size=h.total_size)
    # Huffman fields in a 16-bit-code stream are corrupt too
    hh = _valid_header(n=n, block=block, n_raw=nraw)
    hh.n_sym = 5
    with pytest.raises(pwrel.PwrelError):
        pwrel.read_header_bytes(_bytes(hh), size=hh.total_size)
    hh = _valid_header(n=n, block=block, n_raw=nraw)
    hh.esc_len = 3
    with pytest.raises(pwrel.PwrelError):
        pwrel.read_header_bytes(_bytes(hh), size=hh.total_size)


def _trained_hist(kind, rng):
    h = np.zeros(65536, dtype=np.uint64)
    if kind == "laplace":          # codes of a validation sample: a peak with tails
        c = np.clip(np.round(rng.laplace(32768, 25, 200000)), 0, 65535).astype(np.int64)
        h += np.bincount(c, minlength=65536).astype(np.uint64)
    elif kind == "deep":           # the 16-bit limit binds
        h[100:126] = 2 ** np.arange(1, 27, dtype=np.uint64)
    elif kind == "all_seen":       # no escape: the 32-bit limit
        h[:] = (rng.pareto(1.1, 65536) * 3 + 1).astype(np.uint64)
    elif kind == "one_unseen":     # 65,535 codes plus the escape: every length 16
        h[:] = rng.integers(1, 4, 65536).astype(np.uint64)
        h[777] = 0
    elif kind == "single":
        h[32768] = 99
    elif kind == "empty":
        pass
    else:                          # a few heavy codes and many seen once
        idx = rng.choice(65536, 4000, replace=False)
        h[idx] = 1
        h[idx[:20]] = rng.integers(1000, 100000, 20).astype(np.uint64)
    return h


@pytest.mark.parametrize("kind", ["laplace", "deep", "all_seen", "one_unseen", "single", "empty",
                                  "singletons"])
def test_library_trained_codebook_equals_oracle(kind):
    """The trained codebook of the library (Sec. 4.3: built once from
    validation code counts, an escape for unseen codes) is the oracle's:
    the same length counts, canonical symbols and escape length, bit for
    bit."""
    rng = np.random.default_rng(sum(map(ord, kind)))
    h = _trained_hist(kind, rng)
    cnt, syms, esc = pwrel.huffman_trained_codebook(h).arrays()
    ln, oesc = O.huff_trained_lengths(h)
    ocnt, osyms = O.huff_book(ln)
    assert esc == oesc
    assert np.array_equal(cnt, ocnt)
    assert np.array_equal(syms, osyms)
    if kind == "all_seen":
        assert esc == 0 and int(cnt.sum()) == 65536
    if kind in ("deep", "one_unseen"):
        assert esc > 0 and max(l for l in range(33) if cnt[l]) == 16
