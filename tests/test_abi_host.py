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
    assert b >= 512 + C.sizeof(pwrel.Mlp) + nb + 4 * nb + 2 * n + 4 * n
    assert b < 512 + 4096 + nb + 4 * nb + 2 * n + 4 * n
    assert pwrel.compress_bound((8, 8, 8), 3, 8) == 0


def _valid_header(n=(10, 12), block=4, flags=0, dtype=pwrel.F32, n_raw=3):
    h = pwrel.Header()
    h.magic, h.version, h.dtype, h.ndim = 0x4C455750, 1, dtype, len(n)
    for d, v in enumerate(n):
        h.dims[d] = v
    h.block, h.flags = block, flags
    h.eps, h.w, h.r, h.b_a = 1e-2, 0.0287, 34.8, 0.01435
    h.Lp, h.Ln, h.p_zero, h.b_sign, h.delta = 0.0, 2.0, -4389, 70, 0
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
                   ("delta", -1), ("flags", 64)]
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
