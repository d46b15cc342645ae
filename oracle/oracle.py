"""ctypes front-end of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: only tests/, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It loads
oracle/liboracle.so (built from oracle/pwrel_oracle.c; compiled on first use
if missing) and shares no code with the HIP library.

A network ("model") is passed around as a plain dict of numbers:
    {"alpha": float, "w1": float32[H, K], "b1": float32[H], "v": float32[H],
     "b2": float, "precision": 0 (FP32) | 1 (BF16 operands)}
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

F32, F64 = 0, 1
R = 32768
MAXH, MAXK = 32, 6

OK, EINVAL, ERANGE, ENONFINITE, ENOMEM = 0, -1, -2, -3, -7


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


class _Stats(C.Structure):
    _fields_ = [("abs_min", C.c_double), ("abs_max", C.c_double), ("n", C.c_uint64),
                ("n_zero", C.c_uint64), ("n_neg", C.c_uint64), ("n_nonfinite", C.c_uint64)]


class _Consts(C.Structure):
    _fields_ = [("eps", C.c_double), ("eps0", C.c_double), ("b_a", C.c_double),
                ("w", C.c_double), ("r", C.c_double), ("Lp", C.c_double), ("Ln", C.c_double),
                ("d0", C.c_double), ("p_zero", C.c_int64), ("b_sign", C.c_int64),
                ("n_lo", C.c_int64), ("delta", C.c_int64)]


class _MLP(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("inputs", C.c_int32), ("alpha", C.c_float),
                ("w1", (C.c_float * MAXK) * MAXH), ("b1", C.c_float * MAXH),
                ("v", C.c_float * MAXH), ("b2", C.c_float), ("precision", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.or_det_log2.restype = C.c_double
        L.or_det_log2.argtypes = [C.c_double]
        L.or_det_exp2.restype = C.c_double
        L.or_det_exp2.argtypes = [C.c_double]
        L.or_splitmix64.restype = C.c_uint64
        L.or_splitmix64.argtypes = [C.c_uint64]
        L.or_stats_compute.argtypes = [P, C.c_uint64, C.c_int, C.POINTER(_Stats)]
        L.or_consts_compute.argtypes = [C.POINTER(_Stats), C.c_int, C.c_double, C.POINTER(_Consts)]
        L.or_transform_field.argtypes = [P, C.c_uint64, C.c_int, C.POINTER(_Consts), P]
        L.or_inverse_field.argtypes = [P, C.c_uint64, C.c_int, C.POINTER(_Consts), P]
        L.or_verify.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_encode_p.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.POINTER(_MLP), C.c_int, P]
        L.or_compress.argtypes = [P, P, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                  C.POINTER(_MLP), C.c_int, P, P, P, C.POINTER(C.c_uint64),
                                  C.POINTER(_Consts), P, P]
        L.or_decompress.argtypes = [P, P, C.c_uint64, C.POINTER(_Consts), P, C.c_int, C.c_int,
                                    C.c_int, C.c_int, C.POINTER(_MLP), C.c_int, P, P, P]
        L.or_codes_at.argtypes = [P, P, C.c_int, C.c_int, C.POINTER(_Consts), C.c_int, C.c_int,
                                  C.POINTER(_MLP), C.c_int, P, C.c_uint64, P, P, P, P, P, P, P]
        L.or_block_start.restype = C.c_int64
        L.or_block_start.argtypes = [P, C.c_int, C.c_int, P]
        L.or_mlp_init.argtypes = [C.POINTER(_MLP), C.c_int, C.c_int, C.c_float, C.c_uint64]
        L.or_sample.restype = C.c_int64
        L.or_sample.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int64,
                                C.c_double, C.c_uint64, C.c_int64, P, P, P, P]
        L.or_loss_grad.restype = C.c_double
        L.or_loss_grad.argtypes = [P, C.c_int, C.c_int, C.c_double, P, P, C.c_int64, C.c_double,
                                   C.c_double, P]
        L.or_train_pass.argtypes = [P, C.c_int, C.c_int, C.c_double, P, P, C.c_int64, C.c_double,
                                    C.c_double, C.c_double, C.c_int, C.c_int, P, P,
                                    C.POINTER(C.c_int64)]
        L.or_theta_from_mlp.argtypes = [C.POINTER(_MLP), P]
        L.or_mlp_from_theta.argtypes = [C.POINTER(_MLP), P, C.c_double]
        L.or_val_score.restype = C.c_int64
        L.or_val_score.argtypes = [C.POINTER(_MLP), P, P, C.c_int64]
        L.or_train_rule.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int64,
                                    C.c_double, C.c_uint64,
                                    C.POINTER(_MLP), P, C.c_int, P, C.c_int, C.c_int, C.c_int,
                                    C.POINTER(_MLP), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.or_mlp_eval_many.argtypes = [C.POINTER(_MLP), P, C.c_int64, P]
        L.or_mlp_eval_bf16_many.argtypes = [C.POINTER(_MLP), P, C.c_int64, P, P]
        L.or_mlp_eval_f64_many.argtypes = [C.POINTER(_MLP), P, C.c_int64, P, P]
        L.or_loss_grad_abs.argtypes = [P, C.c_int, C.c_int, C.c_double, P, P, C.c_int64,
                                       C.c_double, C.c_double, P, P]
        L.or_theta_eval_many.argtypes = [P, C.c_int, C.c_int, C.c_double, P, C.c_int64,
                                         C.c_double, P]
        L.or_huff_lengths.argtypes = [P, C.c_int, C.c_int, P]
        L.or_huff_canonical.argtypes = [P, C.c_int, C.c_int, P]
        L.or_huff_encode.restype = C.c_int64
        L.or_huff_encode.argtypes = [P, C.c_int64, P, P, P]
        L.or_huff_decode.restype = C.c_int64
        L.or_huff_decode.argtypes = [P, C.c_int64, C.c_int64, P, C.c_int, C.c_int, P]
        L.or_huff_trained_lengths.argtypes = [P, P]
        L.or_huff_encode_esc.restype = C.c_int64
        L.or_huff_encode_esc.argtypes = [P, C.c_int64, P, P, P]
        L.or_huff_decode_esc.restype = C.c_int64
        L.or_huff_decode_esc.argtypes = [P, C.c_int64, C.c_int64, P, C.c_int, P]
        L.or_table_hist.restype = C.c_int64
        L.or_table_hist.argtypes = [P, P, C.c_int, C.c_int, C.c_double, C.c_uint64, P]
        L.or_bf16_rne.restype = C.c_float
        L.or_bf16_rne.argtypes = [C.c_float]
        L.or_entropy_j.restype = C.c_int64
        L.or_entropy_j.argtypes = [P, C.c_int64]
        L.or_judge_j.restype = C.c_int64
        L.or_judge_j.argtypes = [P, C.c_int64]
        L.or_qlog.restype = C.c_int64
        L.or_qlog.argtypes = [C.c_int64]
        L.or_tcoord.restype = C.c_double
        L.or_tcoord.argtypes = [C.c_double, C.POINTER(_Consts)]
        L.or_tinverse.restype = C.c_double
        L.or_tinverse.argtypes = [C.c_double, C.POINTER(_Consts), C.c_int]
        L.or_openloop_encode.argtypes = [P, P, C.c_int, C.c_int, C.c_double, C.c_int,
                                         C.POINTER(_MLP), C.c_int, C.c_int, P, P, P,
                                         C.POINTER(C.c_uint64), P, C.POINTER(_Consts)]
        L.or_openloop_decode.argtypes = [P, P, C.c_uint64, C.POINTER(_Consts), P, C.c_int,
                                         C.c_int, C.c_int, C.POINTER(_MLP), C.c_int, P, P]
        L.or_openloop_choose_m.argtypes = [P, C.c_double]
        for fn in ("or_sizeof_mlp", "or_sizeof_consts", "or_sizeof_stats"):
            getattr(L, fn).restype = C.c_size_t
        assert L.or_sizeof_mlp() == C.sizeof(_MLP)
        assert L.or_sizeof_consts() == C.sizeof(_Consts)
        assert L.or_sizeof_stats() == C.sizeof(_Stats)
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dtype_code(x):
    if x.dtype == np.float32:
        return F32
    if x.dtype == np.float64:
        return F64
    raise TypeError(f"unsupported dtype {x.dtype}")


def _dims(shape):
    return np.ascontiguousarray(np.array(shape, dtype=np.uint64))


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


# --- models -----------------------------------------------------------------

def _to_c_mlp(model):
    m = _MLP()
    if model is None:
        return None
    w1 = np.asarray(model["w1"], dtype=np.float32)
    H, K = w1.shape if w1.ndim == 2 else (len(model["b1"]), 0)
    m.hidden, m.inputs = H, K
    m.alpha = float(model["alpha"])
    for j in range(H):
        for k in range(K):
            m.w1[j][k] = float(w1[j, k])
        m.b1[j] = float(model["b1"][j])
        m.v[j] = float(model["v"][j])
    m.b2 = float(model["b2"])
    m.precision = int(model.get("precision", 0))
    return m


def _from_c_mlp(m):
    H, K = m.hidden, m.inputs
    w1 = np.zeros((H, K), dtype=np.float32)
    for j in range(H):
        for k in range(K):
            w1[j, k] = m.w1[j][k]
    return {"alpha": float(np.float32(m.alpha)), "w1": w1,
            "b1": np.array([m.b1[j] for j in range(H)], dtype=np.float32),
            "v": np.array([m.v[j] for j in range(H)], dtype=np.float32),
            "b2": float(np.float32(m.b2)), "precision": int(m.precision)}


def mlp_init(ndim, hidden, alpha=0.01, seed=0):
    """Network initialised to reproduce Lorenzo exactly (end of Sec. 4.2)."""
    m = _MLP()
    _check(lib().or_mlp_init(C.byref(m), ndim, hidden, alpha, seed), "mlp_init")
    return _from_c_mlp(m)


def mlp_eval(model, u):
    u = np.ascontiguousarray(u, dtype=np.float32)
    n = u.shape[0]
    y = np.zeros(n, dtype=np.float32)
    m = _to_c_mlp(model)
    lib().or_mlp_eval_many(C.byref(m), _ptr(u), n, _ptr(y))
    return y


def mlp_eval_bf16_ref(model, u):
    u = np.ascontiguousarray(u, dtype=np.float32)
    n = u.shape[0]
    y = np.zeros(n)
    s = np.zeros(n)
    m = _to_c_mlp(model)
    lib().or_mlp_eval_bf16_many(C.byref(m), _ptr(u), n, _ptr(y), _ptr(s))
    return y, s


def mlp_eval_f64(model, u):
    """FP64 value of the network (FP32 weights, inputs as FP32 values) and the
    bound on the error of any BF16-operand evaluation of it (the oracle's
    mlp_bf16_bound): returns (y, bound)."""
    u = np.ascontiguousarray(u, dtype=np.float32)
    n = u.shape[0]
    y = np.zeros(n)
    b = np.zeros(n)
    m = _to_c_mlp(model)
    lib().or_mlp_eval_f64_many(C.byref(m), _ptr(u), n, _ptr(y), _ptr(b))
    return y, b


# --- Huffman stage (Sec. 4.1 coding of the codes) --------------------------------------

HUFF_LMAX = 24


def huff_lengths(hist, lmax=HUFF_LMAX):
    """Optimal code lengths with no codeword longer than lmax (package-merge)."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    ln = np.zeros(hist.size, dtype=np.uint8)
    st = lib().or_huff_lengths(_ptr(hist), hist.size, int(lmax), _ptr(ln))
    if st:
        raise OracleError(st, "huff_lengths")
    return ln


def huff_canonical(lengths, lmax=HUFF_LMAX):
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(ln.size, dtype=np.uint32)
    st = lib().or_huff_canonical(_ptr(ln), ln.size, int(lmax), _ptr(code))
    if st:
        raise OracleError(st, "huff_canonical")
    return code


def huff_encode(codes, lengths, lmax=HUFF_LMAX):
    """Bitstream (uint32 words, MSB first) of the codes and its bit count."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    cw = huff_canonical(ln, lmax)
    nbits = int(ln[codes].astype(np.int64).sum())
    words = np.zeros(max((nbits + 31) // 32, 1), dtype=np.uint32)
    got = lib().or_huff_encode(_ptr(codes), codes.size, _ptr(ln), _ptr(cw), _ptr(words))
    assert got == nbits
    return words, nbits


def huff_decode(words, n, lengths, start=0, lmax=HUFF_LMAX):
    """n codes decoded from bit `start` of the stream; returns (codes, end bit)."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    out = np.zeros(max(int(n), 1), dtype=np.uint16)
    end = lib().or_huff_decode(_ptr(words), int(start), int(n), _ptr(ln), ln.size, int(lmax),
                               _ptr(out))
    if end < 0:
        raise OracleError(-5, "huff_decode")
    return out[:n], end


# --- the codebook of the training phase (Sec. 4.3) ----------------------------

ESC = 65536  # alphabet index of the escape symbol


def huff_trained_lengths(hist):
    """Lengths of the codebook built once from validation code counts: an
    array of 65,537 (the 65,536 codes, then the escape), and the escape's
    length (0 when every code was seen)."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    assert hist.size == 65536
    ln = np.zeros(ESC + 1, dtype=np.uint8)
    esc = lib().or_huff_trained_lengths(_ptr(hist), _ptr(ln))
    if esc < 0:
        raise OracleError(esc, "huff_trained_lengths")
    return ln, int(esc)


def huff_encode_esc(codes, lengths):
    """Bitstream of the codes under a trained codebook (lengths of 65,537);
    returns (words, bit count)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    assert ln.size == ESC + 1
    cw = huff_canonical(ln, 32)
    per = np.where(ln[codes] > 0, ln[codes].astype(np.int64), int(ln[ESC]) + 16)
    nbits = int(per.sum())
    words = np.zeros(max((nbits + 31) // 32, 1), dtype=np.uint32)
    got = lib().or_huff_encode_esc(_ptr(codes), codes.size, _ptr(ln), _ptr(cw), _ptr(words))
    if got < 0:
        raise OracleError(int(got), "huff_encode_esc")
    assert got == nbits
    return words, nbits


def huff_decode_esc(words, n, lengths, start=0):
    """n codes decoded under a trained codebook from bit `start`; returns
    (codes, end bit)."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    assert ln.size == ESC + 1
    out = np.zeros(max(int(n), 1), dtype=np.uint16)
    end = lib().or_huff_decode_esc(_ptr(words), int(start), int(n), _ptr(ln), 32, _ptr(out))
    if end < 0:
        raise OracleError(-5, "huff_decode_esc")
    return out[:n], end


def huff_book(lengths):
    """The stream form of a codebook: count[0..32] (codewords per length) and
    the symbols in canonical order (by length, then value); the escape, the
    last symbol of its length, is listed as 0."""
    ln = np.asarray(lengths)
    count = np.bincount(ln[ln > 0], minlength=33).astype(np.uint32)
    syms = [s for L in range(1, 33) for s in np.flatnonzero(ln == L)]
    return count, np.array([0 if s == ESC else s for s in syms], dtype=np.uint16)


def table_hist(codes, shape, B, frac, seed):
    """Code counts of the table's validation blocks (Sec. 4.3): block b of
    the stream order is one iff u01(splitmix64(seed ^ b)) < frac; codes of
    the whole field in stream order.  Returns (hist[65536], number of
    blocks)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    dims = _dims(shape)
    hist = np.zeros(65536, dtype=np.uint64)
    nsel = lib().or_table_hist(_ptr(codes), _ptr(dims), len(shape), int(B), float(frac),
                               int(seed), _ptr(hist))
    if nsel < 0:
        raise OracleError(-1, "table_hist")
    return hist, int(nsel)


# --- deterministic math -------------------------------------------------------

def det_log2(x):
    f = lib().or_det_log2
    if np.isscalar(x):
        return f(float(x))
    return np.array([f(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))


def det_exp2(t):
    f = lib().or_det_exp2
    if np.isscalar(t):
        return f(float(t))
    return np.array([f(float(v)) for v in np.ravel(t)]).reshape(np.shape(t))


def splitmix64(state):
    return int(lib().or_splitmix64(int(state) & 0xFFFFFFFFFFFFFFFF))


def bf16_rne(f):
    return float(lib().or_bf16_rne(float(f)))


# --- statistics / constants / transform ----------------------------------------

def stats(x):
    x = np.ascontiguousarray(x)
    s = _Stats()
    st = lib().or_stats_compute(_ptr(x), x.size, _dtype_code(x), C.byref(s))
    return st, {k: getattr(s, k) for k, _ in _Stats._fields_}


def _consts_struct(c):
    s = _Consts()
    for k, _ in _Consts._fields_:
        setattr(s, k, c[k])
    return s


def consts(x, eps):
    """Constants of Step 2 for field x (dict)."""
    x = np.ascontiguousarray(x)
    st, _ = stats(x)
    _check(st, "stats")
    s = _Stats()
    lib().or_stats_compute(_ptr(x), x.size, _dtype_code(x), C.byref(s))
    c = _Consts()
    _check(lib().or_consts_compute(C.byref(s), _dtype_code(x), float(eps), C.byref(c)), "consts")
    return {k: getattr(c, k) for k, _ in _Consts._fields_}


def transform_field(x, c):
    x = np.ascontiguousarray(x)
    p = np.zeros(x.shape, dtype=np.int32)
    cs = _consts_struct(c)
    _check(lib().or_transform_field(_ptr(x), x.size, _dtype_code(x), C.byref(cs), _ptr(p)),
           "transform")
    return p


def inverse_field(p, c, dtype):
    p = np.ascontiguousarray(p, dtype=np.int32)
    out = np.zeros(p.shape, dtype=dtype)
    cs = _consts_struct(c)
    lib().or_inverse_field(_ptr(p), p.size, _dtype_code(out), C.byref(cs), _ptr(out))
    return out


def verify(x, xh, eps):
    return bool(lib().or_verify(float(x), float(xh), float(eps)))


# --- compression ----------------------------------------------------------------

MODE_LORENZO, MODE_PLAIN, MODE_LEARNED = 0, 1, 2


def nblocks(shape, B):
    n = 1
    for d in shape:
        n *= -(-d // B)
    return n


def compress(x, eps, B, model=None, mode=MODE_PLAIN, independent=False):
    """Oracle compression; returns dict(codes, counts, raw, consts, flags, p)."""
    x = np.ascontiguousarray(x)
    dims = _dims(x.shape)
    N, nb = x.size, nblocks(x.shape, B)
    codes = np.zeros(N, dtype=np.uint16)
    counts = np.zeros(nb, dtype=np.uint32)
    raw = np.zeros(N, dtype=x.dtype)
    flags = np.zeros(nb, dtype=np.uint8)
    p = np.zeros(x.shape, dtype=np.int32)
    nraw = C.c_uint64(0)
    c = _Consts()
    m = _to_c_mlp(model)
    st = lib().or_compress(_ptr(x), _ptr(dims), x.ndim, _dtype_code(x), float(eps), B,
                           int(bool(independent)), C.byref(m) if m is not None else None, mode,
                           _ptr(codes), _ptr(counts), _ptr(raw), C.byref(nraw), C.byref(c),
                           _ptr(flags), _ptr(p))
    _check(st, "compress")
    return {"codes": codes, "counts": counts, "raw": raw[:nraw.value].copy(),
            "consts": {k: getattr(c, k) for k, _ in _Consts._fields_}, "flags": flags, "p": p}


def decompress(codes, raw, c, shape, dtype, B, model=None, mode=MODE_PLAIN, flags=None,
               independent=False):
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    raw = np.ascontiguousarray(raw, dtype=dtype)
    dims = _dims(shape)
    xh = np.zeros(shape, dtype=dtype)
    p = np.zeros(shape, dtype=np.int32)
    cs = _consts_struct(c)
    m = _to_c_mlp(model)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    st = lib().or_decompress(_ptr(codes), _ptr(raw), raw.size, C.byref(cs), _ptr(dims),
                             len(shape), _dtype_code(xh), B, int(bool(independent)),
                             C.byref(m) if m is not None else None, mode, _ptr(fl), _ptr(xh),
                             _ptr(p))
    _check(st, "decompress")
    return xh, p


def codes_at(x, c, B, idx, model=None, mode=MODE_PLAIN, independent=False):
    """Code, stream position and grid value of selected points (C-order
    linear indices), each computed from the field alone."""
    x = np.ascontiguousarray(x)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    dims = _dims(x.shape)
    n = idx.size
    codes = np.zeros(n, dtype=np.uint16)
    pos = np.zeros(n, dtype=np.uint64)
    p = np.zeros(n, dtype=np.int32)
    yref = np.zeros(n)
    slack = np.zeros(n)
    y64 = np.zeros(n)
    bound = np.zeros(n)
    cs = _consts_struct(c)
    m = _to_c_mlp(model)
    st = lib().or_codes_at(_ptr(x), _ptr(dims), x.ndim, _dtype_code(x), C.byref(cs), B,
                           int(bool(independent)), C.byref(m) if m is not None else None, mode,
                           _ptr(idx), n, _ptr(codes), _ptr(pos), _ptr(p), _ptr(yref),
                           _ptr(slack), _ptr(y64), _ptr(bound))
    _check(st, "codes_at")
    return {"codes": codes, "pos": pos, "p": p, "yref": yref, "slack": slack, "y64": y64,
            "bound": bound}


def encode_p(p, B, model=None, use_net=True, independent=False):
    p = np.ascontiguousarray(p, dtype=np.int32)
    dims = _dims(p.shape)
    codes = np.zeros(p.size, dtype=np.uint16)
    m = _to_c_mlp(model)
    _check(lib().or_encode_p(_ptr(p), _ptr(dims), p.ndim, B, int(bool(independent)),
                             C.byref(m) if m is not None else None, int(bool(use_net)),
                             _ptr(codes)), "encode_p")
    return codes


def block_start(shape, B, bc):
    dims = _dims(shape)
    bc = np.ascontiguousarray(np.array(bc, dtype=np.int64))
    return int(lib().or_block_start(_ptr(dims), len(shape), B, _ptr(bc)))


def entropy_j(codes):
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    return int(lib().or_entropy_j(_ptr(codes), codes.size))


def judge_j(codes):
    """Per-block judge score of a block's codes: J of their full multiset
    (n q(n) - J = 2^32 x the block's code entropy in bits)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    return int(lib().or_judge_j(_ptr(codes), codes.size))


def qlog(c):
    return int(lib().or_qlog(int(c)))


# --- training -------------------------------------------------------------------

def sample(p, c, B, rho, seed, independent=False):
    """Training pairs drawn from grid field p (constants c give the ranges)."""
    p = np.ascontiguousarray(p, dtype=np.int32)
    dims = _dims(p.shape)
    K = (1 << p.ndim) - 2
    L = lib()
    pz, bs = int(c["p_zero"]), int(c["b_sign"])
    n = L.or_sample(_ptr(p), _ptr(dims), p.ndim, B, int(bool(independent)), pz, bs, float(rho),
                    seed, 0, None, None, None, None)
    u = np.zeros((max(n, 1), K), dtype=np.int32)
    t = np.zeros(max(n, 1), dtype=np.int32)
    iv = np.zeros(max(n, 1), dtype=np.uint8)
    ix = np.zeros(max(n, 1), dtype=np.uint64)
    L.or_sample(_ptr(p), _ptr(dims), p.ndim, B, int(bool(independent)), pz, bs, float(rho),
                seed, n, _ptr(u), _ptr(t), _ptr(iv), _ptr(ix))
    return {"u": u[:n], "t": t[:n], "is_val": iv[:n].astype(bool), "idx": ix[:n]}


def theta_from_model(model):
    m = _to_c_mlp(model)
    H, K = m.hidden, m.inputs
    th = np.zeros(H * K + 2 * H + 1)
    lib().or_theta_from_mlp(C.byref(m), _ptr(th))
    return th


def model_from_theta(template, theta, sigma):
    m = _to_c_mlp(template)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    lib().or_mlp_from_theta(C.byref(m), _ptr(th), float(sigma))
    return _from_c_mlp(m)


def loss_grad(theta, H, K, alpha, u, t, sigma, lam):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    g = np.zeros_like(theta)
    loss = lib().or_loss_grad(_ptr(theta), H, K, float(alpha), _ptr(u), _ptr(t), t.size,
                              float(sigma), float(lam), _ptr(g))
    return loss, g


def loss_grad_abs(theta, H, K, alpha, u, t, sigma, lam):
    """Per-component magnitudes behind loss_grad's gradient: (gabs, gres) --
    the sum of |terms| and the residual magnitudes times |dy/dtheta| (see
    or_loss_grad_abs)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    g = np.zeros_like(theta)
    r = np.zeros_like(theta)
    lib().or_loss_grad_abs(_ptr(theta), H, K, float(alpha), _ptr(u), _ptr(t), t.size,
                           float(sigma), float(lam), _ptr(g), _ptr(r))
    return g, r


def theta_eval(theta, H, K, alpha, u, sigma):
    """FP64 output of scaled-domain parameters theta for inputs u / sigma."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, K) if K else \
        np.zeros((np.shape(u)[0], 0))
    y = np.zeros(u.shape[0])
    lib().or_theta_eval_many(_ptr(theta), H, K, float(alpha), _ptr(u), u.shape[0],
                             float(sigma), _ptr(y))
    return y


def train_pass(theta, H, K, alpha, u, t, sigma, lam, lr, batch, opt, adam_m=None, adam_v=None,
               step=0):
    theta = np.array(theta, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    am = np.zeros_like(theta) if adam_m is None else np.array(adam_m, dtype=np.float64)
    av = np.zeros_like(theta) if adam_v is None else np.array(adam_v, dtype=np.float64)
    s = C.c_int64(step)
    _check(lib().or_train_pass(_ptr(theta), H, K, float(alpha), _ptr(u), _ptr(t), t.size,
                               float(sigma), float(lam), float(lr), int(batch), int(opt),
                               _ptr(am), _ptr(av), C.byref(s)), "train_pass")
    return theta, am, av, s.value


def val_score(model, u, t):
    u = np.ascontiguousarray(u, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    m = _to_c_mlp(model)
    return int(lib().or_val_score(C.byref(m), _ptr(u), _ptr(t), t.size))


DEFAULT_LRS = (3e-2, 1e-2, 3e-3)
DEFAULT_LAMBDAS = (0.0, 1e-5, 1e-4)


def train_rule(p, c, B, init, rho=0.10, seed=0, lrs=DEFAULT_LRS, lambdas=DEFAULT_LAMBDAS,
               batch=256, opt=0, independent=False):
    """The oracle's training rule on grid field p with constants c; returns
    (model, chosen_index, n_train, n_val)."""
    p = np.ascontiguousarray(p, dtype=np.int32)
    dims = _dims(p.shape)
    lr = np.ascontiguousarray(np.array(lrs, dtype=np.float64))
    lm = np.ascontiguousarray(np.array(lambdas, dtype=np.float64))
    mi = _to_c_mlp(init)
    out = _MLP()
    ntr, nva = C.c_int64(0), C.c_int64(0)
    st = lib().or_train_rule(_ptr(p), _ptr(dims), p.ndim, B, int(bool(independent)),
                             int(c["p_zero"]), int(c["b_sign"]), float(rho), seed, C.byref(mi), _ptr(lr), lr.size, _ptr(lm),
                             lm.size, batch, opt, C.byref(out), C.byref(ntr), C.byref(nva))
    if st < 0:
        raise OracleError(st, "train_rule")
    return _from_c_mlp(out), st, ntr.value, nva.value


# --- open-loop mode (the paper's literal data selection; Sec. 4.3, 4.4) ------------------------

def tcoord(x, c):
    """Continuous grid coordinate of each value of x (before rounding)."""
    cs = _consts_struct(c)
    xf = np.asarray(x, dtype=np.float64).ravel()
    return np.array([lib().or_tcoord(float(v), C.byref(cs)) for v in xf]).reshape(np.shape(x))


def tinverse(t, c, dtype):
    cs = _consts_struct(c)
    dc = 0 if np.dtype(dtype) == np.float32 else 1
    tf = np.asarray(t, dtype=np.float64).ravel()
    out = np.array([lib().or_tinverse(float(v), C.byref(cs), dc) for v in tf])
    return out.astype(dtype).reshape(np.shape(t))


def openloop_encode(x, eps, B, model=None, mbits=16, gap=0):
    """Open-loop compression (independent blocks); returns dict(codes,
    counts, raw, hist, consts)."""
    x = np.ascontiguousarray(x)
    dims = _dims(x.shape)
    N, nb = x.size, nblocks(x.shape, B)
    codes = np.zeros(N, dtype=np.uint16)
    counts = np.zeros(nb, dtype=np.uint32)
    raw = np.zeros(N, dtype=x.dtype)
    hist = np.zeros(18, dtype=np.uint64)
    nraw = C.c_uint64(0)
    c = _Consts()
    m = _to_c_mlp(model)
    st = lib().or_openloop_encode(_ptr(x), _ptr(dims), x.ndim, _dtype_code(x), float(eps), B,
                                  C.byref(m) if m is not None else None, int(mbits), int(gap),
                                  _ptr(codes), _ptr(counts), _ptr(raw), C.byref(nraw),
                                  _ptr(hist), C.byref(c))
    _check(st, "openloop_encode")
    return {"codes": codes, "counts": counts, "raw": raw[:nraw.value].copy(), "hist": hist,
            "consts": {k: getattr(c, k) for k, _ in _Consts._fields_}}


def openloop_decode(codes, raw, c, shape, dtype, B, model=None, mbits=16):
    """Open-loop decompression; returns (x^, reconstructed coordinates)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    raw = np.ascontiguousarray(raw, dtype=dtype)
    dims = _dims(shape)
    xh = np.zeros(shape, dtype=dtype)
    t = np.zeros(shape, dtype=np.float64)
    cs = _consts_struct(c)
    m = _to_c_mlp(model)
    st = lib().or_openloop_decode(_ptr(codes), _ptr(raw), raw.size, C.byref(cs), _ptr(dims),
                                  len(shape), _dtype_code(xh), B,
                                  C.byref(m) if m is not None else None, int(mbits), _ptr(xh),
                                  _ptr(t))
    _check(st, "openloop_decode")
    return xh, t


def openloop_choose_m(hist, eps):
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return int(lib().or_openloop_choose_m(_ptr(h), float(eps)))


def openloop_report(x, xh, eps):
    """Violations of the PW_REL bound (sign and zero included) and the
    largest relative error over the non-zero values."""
    xd, hd = np.asarray(x, np.float64).ravel(), np.asarray(xh, np.float64).ravel()
    nz = xd != 0
    bad = np.zeros(xd.size, dtype=bool)
    bad[~nz] = hd[~nz] != 0
    with np.errstate(invalid="ignore", over="ignore"):
        rel = np.where(nz, np.abs(xd - hd) / np.where(nz, np.abs(xd), 1.0), 0.0)
    bad[nz] = (np.signbit(xd[nz]) != np.signbit(hd[nz])) | (hd[nz] == 0) | \
        ~(np.abs(xd[nz] - hd[nz]) <= eps * np.abs(xd[nz]))
    return {"violations": int(bad.sum()), "max_rel": float(np.max(rel)) if rel.size else 0.0}
