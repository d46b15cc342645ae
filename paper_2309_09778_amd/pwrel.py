"""Thin ctypes binding of libpwrel.so (C ABI in include/pwrel.h).

Argument marshalling only: every step of compression and decompression runs
in the library's HIP kernels.  PyTorch provides device memory (tensors) and
streams (torch.cuda.current_stream()).  Importing this module does not touch
the GPU; loading the library fails loudly if it has not been built.

A network ("model") is a plain dict:
    {"alpha": float, "w1": float32[H, K], "b1": float32[H], "v": float32[H],
     "b2": float, "precision": 0 (FP32 vector ALU) | 1 (BF16 matrix cores)}
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwrel.so")

F32, F64 = 0, 1
OK, EINVAL, ERANGE, ENONFINITE, ENOSPC, ECORRUPT, EHIP, ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7
HF_NET, HF_JUDGE, HF_INDEPENDENT, HF_HUFFMAN = 1, 2, 4, 8
HUFF_MAX_LEN = 32
BATCH_TILES = 3
HEADER_BYTES = 512
MAXH, MAXK = 32, 6
R = 32768


class PwrelError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pwrel status {status}: {msg}")
        self.status = status


class Mlp(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("inputs", C.c_int32), ("alpha", C.c_float),
                ("w1", (C.c_float * MAXK) * MAXH), ("b1", C.c_float * MAXH),
                ("v", C.c_float * MAXH), ("b2", C.c_float), ("precision", C.c_int32)]


class Codebook(C.Structure):
    """pwrel_codebook: a trained Huffman codebook (count[l] per length, the
    symbols in canonical order, the escape's length or 0)."""
    _fields_ = [("count", C.c_uint32 * 33), ("n_sym", C.c_uint32), ("esc_len", C.c_uint32),
                ("syms", C.c_uint16 * 65536)]

    def arrays(self):
        """(count[33], syms[n_sym], esc_len) as numpy arrays."""
        cnt = np.frombuffer(self.count, dtype=np.uint32).copy()
        syms = np.frombuffer(self.syms, dtype=np.uint16)[:self.n_sym].copy()
        return cnt, syms, int(self.esc_len)


class Options(C.Structure):
    _fields_ = [("use_net", C.c_int32), ("judge", C.c_int32),
                ("independent_blocks", C.c_int32), ("entropy", C.c_int32),
                ("codebook", C.POINTER(Codebook))]


class Header(C.Structure):
    _fields_ = [("magic", C.c_uint32), ("version", C.c_uint32), ("dtype", C.c_int32),
                ("ndim", C.c_int32), ("dims", C.c_uint64 * 3), ("block", C.c_int32),
                ("flags", C.c_int32), ("eps", C.c_double), ("eps0", C.c_double),
                ("b_a", C.c_double), ("w", C.c_double), ("r", C.c_double), ("Lp", C.c_double),
                ("Ln", C.c_double), ("d0", C.c_double), ("p_zero", C.c_int64),
                ("b_sign", C.c_int64), ("n_lo", C.c_int64), ("delta", C.c_int64),
                ("n", C.c_uint64), ("nblocks", C.c_uint64), ("n_raw", C.c_uint64),
                ("off_model", C.c_uint64), ("off_bflags", C.c_uint64),
                ("off_counts", C.c_uint64), ("off_codes", C.c_uint64), ("off_raw", C.c_uint64),
                ("total_size", C.c_uint64), ("abs_min", C.c_double), ("abs_max", C.c_double),
                ("n_zero", C.c_uint64), ("n_neg", C.c_uint64), ("status", C.c_int32),
                ("esc_len", C.c_uint32), ("off_huff", C.c_uint64), ("off_sizes", C.c_uint64),
                ("off_bits", C.c_uint64), ("n_bits", C.c_uint64), ("n_sym", C.c_uint32),
                ("size_bytes", C.c_uint32), ("p_max", C.c_int64)]


MAX_CANDIDATES = 17
FAST_LOG2_ERR = 2.0 ** -20  # PWREL_FAST_LOG2_ERR
FAST_EXP2_ERR = 2.0 ** -20  # PWREL_FAST_EXP2_ERR


class FieldDesc(C.Structure):
    _fields_ = [("d_field", C.c_void_p), ("dims", C.c_uint64 * 3), ("ndim", C.c_int32),
                ("reserved", C.c_int32), ("d_out", C.c_void_p), ("out_capacity", C.c_uint64)]


class OpenloopReport(C.Structure):
    _fields_ = [("n_raw", C.c_uint64), ("violations", C.c_uint64),
                ("max_rel_error", C.c_double), ("hist", C.c_uint64 * 18), ("mbits", C.c_int32),
                ("gap", C.c_int32)]


class TrainOptions(C.Structure):
    _fields_ = [("rho", C.c_double), ("seed", C.c_uint64), ("hidden", C.c_int32),
                ("epochs", C.c_int32), ("batch", C.c_int32), ("n_lr", C.c_int32),
                ("n_lambda", C.c_int32), ("independent_blocks", C.c_int32),
                ("lr", C.c_double * 4), ("lambda_", C.c_double * 4), ("alpha", C.c_float),
                ("precision", C.c_int32)]


class TrainReport(C.Structure):
    _fields_ = [("n_train", C.c_uint64), ("n_val", C.c_uint64), ("sigma", C.c_double),
                ("chosen", C.c_int32), ("n_candidates", C.c_int32),
                ("val_score", C.c_int64 * MAX_CANDIDATES), ("ms_sample", C.c_double),
                ("ms_train", C.c_double), ("ms_select", C.c_double)]


DEFAULT_LRS = (3e-2, 1e-2, 3e-3)
DEFAULT_LAMBDAS = (0.0, 1e-5, 1e-4)

# every symbol the header declares, with its signature
_P = C.c_void_p
_SIGS = {
    "pwrel_create": (C.c_int, [C.POINTER(_P), C.c_int]),
    "pwrel_destroy": (None, [_P]),
    "pwrel_last_error": (C.c_char_p, [_P]),
    "pwrel_status_string": (C.c_char_p, [C.c_int]),
    "pwrel_check_args": (C.c_int, [_P, C.c_int, C.c_int, C.c_double, C.c_int]),
    "pwrel_compress_bound": (C.c_uint64, [_P, C.c_int, C.c_int, C.c_int]),
    "pwrel_compress": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int,
                                 C.POINTER(Mlp), C.POINTER(Options), _P, C.c_uint64,
                                 C.POINTER(C.c_uint64), _P]),
    "pwrel_compress_noalloc": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int,
                                         C.POINTER(Mlp), C.POINTER(Options), _P, C.c_uint64,
                                         C.POINTER(C.c_uint64), _P]),
    "pwrel_compress_batch": (C.c_int, [_P, C.c_int, C.POINTER(FieldDesc), C.c_int, C.c_double,
                                       _P, C.POINTER(C.POINTER(Mlp)), C.POINTER(Options), _P,
                                       _P]),
    "pwrel_batch_set_tiles": (C.c_int, [_P, _P]),
    "pwrel_batch_get_tiles": (C.c_int, [_P, _P, _P]),
    "pwrel_compress_batch_tune": (C.c_int, [_P, C.c_int, C.POINTER(FieldDesc), C.c_int,
                                            C.c_double, _P, C.POINTER(C.POINTER(Mlp)),
                                            C.POINTER(Options), _P, C.c_int, _P, _P, _P]),
    "pwrel_openloop": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int,
                                 C.POINTER(Mlp), C.c_int, C.c_int, _P, _P, _P, C.c_uint64, _P,
                                 C.POINTER(OpenloopReport), _P]),
    "pwrel_decompress": (C.c_int, [_P, _P, C.c_uint64, _P, _P, C.c_int, C.c_int, _P]),
    "pwrel_read_header": (C.c_int, [_P, C.c_uint64, C.POINTER(Header)]),
    "pwrel_compress_raw": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int,
                                     C.POINTER(Mlp), C.POINTER(Options), _P, _P, _P, _P,
                                     C.c_uint64, C.POINTER(Header), _P]),
    "pwrel_model_save": (C.c_int, [C.POINTER(Mlp), _P, C.c_uint64, C.POINTER(C.c_uint64)]),
    "pwrel_model_load": (C.c_int, [_P, C.c_uint64, C.POINTER(Mlp)]),
    "pwrel_stream_model": (C.c_int, [_P, _P, C.c_uint64, C.POINTER(Mlp), _P]),
    "pwrel_transform": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, _P,
                                  C.POINTER(Header), _P]),
    "pwrel_encode_grid": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.POINTER(Mlp),
                                    C.POINTER(Options), _P, _P]),
    "pwrel_detmath": (C.c_int, [_P, _P, _P, _P, C.c_uint64, _P]),
    "pwrel_histogram": (C.c_int, [_P, _P, C.c_uint64, _P, _P]),
    "pwrel_huffman_bits": (C.c_uint64, [_P, C.POINTER(C.c_uint32)]),
    "pwrel_huffman_codebook": (C.c_int, [_P, _P, _P, C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint64)]),
    "pwrel_huffman_trained_codebook": (C.c_int, [_P, C.POINTER(Codebook)]),
    "pwrel_compress_datablocks": (C.c_int, [_P, _P, _P, C.c_double, C.c_int, C.POINTER(Mlp),
                                            C.POINTER(Options), _P, C.c_uint64, _P,
                                            C.POINTER(C.c_uint64), _P]),
    "pwrel_decompress_datablocks": (C.c_int, [_P, _P, C.c_uint64, _P, _P, _P, C.c_int, _P]),
    "pwrel_train_codebook": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int,
                                       C.POINTER(Mlp), C.POINTER(Options), C.c_double,
                                       C.c_uint64, C.POINTER(Codebook), _P]),
    "pwrel_mlp_init": (C.c_int, [C.POINTER(Mlp), C.c_int, C.c_int, C.c_float, C.c_uint64]),
    "pwrel_set_profiling": (C.c_int, [_P, C.c_int]),
    "pwrel_phase_times": (C.c_int, [_P, _P, C.c_int]),
    "pwrel_fastmath_check": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double), _P]),
    "pwrel_train": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int,
                              C.POINTER(TrainOptions), C.POINTER(Mlp), C.POINTER(Mlp),
                              C.POINTER(TrainReport), _P]),
    "pwrel_sample": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                               C.c_double, C.c_uint64, _P, _P, _P, _P, C.c_uint64,
                               C.POINTER(C.c_uint64), _P]),
    "pwrel_loss_grad": (C.c_int, [_P, _P, C.c_int, C.c_int, C.c_float, _P, _P, C.c_uint64,
                                  C.c_double, C.c_double, _P, C.POINTER(C.c_float), _P]),
    "pwrel_train_pairs": (C.c_int, [_P, _P, _P, C.c_uint64, C.c_int, C.c_int, C.c_float,
                                    C.c_double, _P, C.c_int, _P, _P, C.c_int, C.c_int, _P,
                                    _P]),
}
PHASES = ("stats+consts", "compress", "scan+scatter+header", "decode_scan", "decode_levels",
          "decode_raw_grid", "decode_inverse")

_lib = None


def lib():
    """Load libpwrel.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        assert C.sizeof(Header) <= HEADER_BYTES
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


# --- helpers --------------------------------------------------------------------

def _dims(shape):
    return (C.c_uint64 * len(shape))(*[int(s) for s in shape])


def _dtype_code(tdtype):
    import torch
    if tdtype == torch.float32:
        return F32
    if tdtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {tdtype}")


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def model_struct(model):
    """The C struct of a model dict (an Mlp passes through unchanged)."""
    if model is None or isinstance(model, Mlp):
        return model
    m = Mlp()
    w1 = np.asarray(model["w1"], dtype=np.float32)
    H = len(model["b1"])
    K = w1.shape[1] if w1.ndim == 2 else 0
    if H > MAXH or K > MAXK:
        raise ValueError(f"network {H}x{K} exceeds {MAXH}x{MAXK}")
    m.hidden, m.inputs = H, K
    m.alpha = float(model["alpha"])
    # whole arrays at once (zero padded to the struct's fixed sizes)
    w1p = np.zeros((MAXH, MAXK), dtype=np.float32)
    w1p[:H, :K] = w1.reshape(H, K)
    b1p = np.zeros(MAXH, dtype=np.float32)
    b1p[:H] = np.asarray(model["b1"], dtype=np.float32)
    vp = np.zeros(MAXH, dtype=np.float32)
    vp[:H] = np.asarray(model["v"], dtype=np.float32)
    C.memmove(C.addressof(m.w1), w1p.ctypes.data, C.sizeof(m.w1))
    C.memmove(C.addressof(m.b1), b1p.ctypes.data, C.sizeof(m.b1))
    C.memmove(C.addressof(m.v), vp.ctypes.data, C.sizeof(m.v))
    m.b2 = float(model["b2"])
    m.precision = int(model.get("precision", 0))
    return m


def model_dict(m):
    H, K = m.hidden, m.inputs
    w1 = np.array([[m.w1[j][k] for k in range(K)] for j in range(H)],
                  dtype=np.float32).reshape(H, K)
    return {"alpha": float(np.float32(m.alpha)), "w1": w1,
            "b1": np.array([m.b1[j] for j in range(H)], dtype=np.float32),
            "v": np.array([m.v[j] for j in range(H)], dtype=np.float32),
            "b2": float(np.float32(m.b2)), "precision": int(m.precision)}


def mlp_init(ndim, hidden, alpha=0.01, seed=0):
    m = Mlp()
    st = lib().pwrel_mlp_init(C.byref(m), ndim, hidden, alpha, seed)
    if st:
        raise PwrelError(st, "mlp_init")
    return model_dict(m)


def header_dict(h):
    out = {}
    for name, _ in Header._fields_:
        v = getattr(h, name)
        out[name] = list(v) if name == "dims" else v
    return out


def check_args(shape, dtype_code, eps, block):
    return lib().pwrel_check_args(_dims(shape), len(shape), dtype_code, float(eps), int(block))


def compress_bound(shape, dtype_code, block):
    return int(lib().pwrel_compress_bound(_dims(shape), len(shape), dtype_code, int(block)))


def read_header_bytes(buf, size=None):
    """Validate a header held in host memory; `size` is the whole stream's
    length (default: len(buf)).  Returns a dict."""
    raw = bytes(buf)
    h = Header()
    b = C.create_string_buffer(raw, max(len(raw), HEADER_BYTES))
    st = lib().pwrel_read_header(C.cast(b, _P), len(raw) if size is None else int(size),
                                 C.byref(h))
    if st:
        raise PwrelError(st, "read_header")
    return header_dict(h)


def model_save(model):
    """Serialise a network (dict or Mlp) to bytes (pwrel_model_save)."""
    m = model_struct(model)
    size = C.c_uint64(0)
    st = lib().pwrel_model_save(C.byref(m), None, 0, C.byref(size))
    if st not in (OK, ENOSPC):
        raise PwrelError(st, "model_save")
    buf = C.create_string_buffer(size.value)
    st = lib().pwrel_model_save(C.byref(m), C.cast(buf, _P), size.value, C.byref(size))
    if st:
        raise PwrelError(st, "model_save")
    return buf.raw[:size.value]


def model_load(data):
    """Parse bytes written by model_save into a network dict (pwrel_model_load)."""
    data = bytes(data)
    buf = C.create_string_buffer(data, max(len(data), 1))
    m = Mlp()
    st = lib().pwrel_model_load(C.cast(buf, _P), len(data), C.byref(m))
    if st:
        raise PwrelError(st, "model_load")
    return model_dict(m)


def huffman_bits(hist):
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    assert hist.size == 65536
    ml = C.c_uint32(0)
    bits = lib().pwrel_huffman_bits(hist.ctypes.data_as(_P), C.byref(ml))
    return int(bits), int(ml.value)


def huffman_codebook(hist):
    """The library's codebook for a 65,536-bin histogram: (count[33], syms in
    canonical order, total coded bits)."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    assert hist.size == 65536
    cnt = np.zeros(HUFF_MAX_LEN + 1, dtype=np.uint32)
    syms = np.zeros(65536, dtype=np.uint16)
    ns, nb = C.c_uint32(0), C.c_uint64(0)
    st = lib().pwrel_huffman_codebook(hist.ctypes.data_as(_P), cnt.ctypes.data_as(_P),
                                      syms.ctypes.data_as(_P), C.byref(ns), C.byref(nb))
    if st:
        raise PwrelError(st, "huffman_codebook")
    return cnt, syms[:ns.value].copy(), int(nb.value)


def huffman_trained_codebook(hist):
    """The library's trained codebook (Sec. 4.3) of a 65,536-bin validation
    code histogram, as a Codebook."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    assert hist.size == 65536
    cb = Codebook()
    st = lib().pwrel_huffman_trained_codebook(hist.ctypes.data_as(_P), C.byref(cb))
    if st:
        raise PwrelError(st, "huffman_trained_codebook")
    return cb


def codebook_lengths(count, syms):
    """Per-symbol codeword lengths (65,536 entries, 0 = unused) of a codebook
    given as length counts and canonical-order symbols."""
    ln = np.zeros(65536, dtype=np.uint8)
    i = 0
    for l in range(1, len(count)):
        c = int(count[l])
        ln[np.asarray(syms[i:i + c], dtype=np.int64)] = l
        i += c
    return ln


# --- context ----------------------------------------------------------------------

class Context:
    """A pwrel context on one GPU (owns the device workspace)."""

    def __init__(self, device=0):
        self._L = lib()
        self.device = device
        h = _P()
        st = self._L.pwrel_create(C.byref(h), device)
        if st:
            raise PwrelError(st, "pwrel_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self._L.pwrel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st:
            msg = self._L.pwrel_last_error(self.h)
            raise PwrelError(st, f"{what}: {msg.decode() if msg else ''}")

    # codec -------------------------------------------------------------------
    def compress(self, x, eps, block=8, model=None, use_net=True, judge=False,
                 independent=False, entropy=False, out=None, stream=None, codebook=None):
        """Compress a contiguous CUDA tensor; returns a uint8 CUDA tensor view.
        entropy=True: the codes are Huffman coded in the stream; codebook (a
        Codebook, implies entropy): that trained table instead of one built
        from the field's histogram."""
        import torch
        assert x.is_cuda and x.is_contiguous()
        dt = _dtype_code(x.dtype)
        cap = compress_bound(x.shape, dt, block)
        if cap == 0:
            raise PwrelError(EINVAL, "bad shape/block")
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        m = model_struct(model) if use_net else None
        opt = Options(int(bool(use_net)), int(bool(judge)), int(bool(independent)),
                      int(bool(entropy) or codebook is not None))
        if codebook is not None:
            opt.codebook = C.pointer(codebook)
        size = C.c_uint64(0)
        st = self._L.pwrel_compress(self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(),
                                    dt, float(eps), int(block),
                                    C.byref(m) if m is not None else None, C.byref(opt),
                                    C.c_void_p(out.data_ptr()), out.numel(), C.byref(size),
                                    _stream(stream))
        self._check(st, "compress")
        return out[:size.value]

    def compress_noalloc(self, x, eps, block=8, model=None, use_net=True, judge=False,
                         independent=False, out=None, stream=None):
        """pwrel_compress_noalloc: as compress(), with the library's static
        device scratch instead of the context's workspace (the output tensor
        is the caller's: pass `out` to allocate nothing at all)."""
        import torch
        assert x.is_cuda and x.is_contiguous()
        dt = _dtype_code(x.dtype)
        cap = compress_bound(x.shape, dt, block)
        if out is None:
            out = torch.empty(max(cap, 1), dtype=torch.uint8, device=x.device)
        m = model_struct(model) if use_net else None
        opt = Options(int(bool(use_net)), int(bool(judge)), int(bool(independent)), 0)
        size = C.c_uint64(0)
        st = self._L.pwrel_compress_noalloc(
            self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(), dt, float(eps),
            int(block), C.byref(m) if m is not None else None, C.byref(opt),
            C.c_void_p(out.data_ptr()), out.numel(), C.byref(size), _stream(stream))
        self._check(st, "compress_noalloc")
        return out[:size.value]

    def batch_request(self, xs, eps, models=None, use_net=True, judge=False,
                      independent=False, blocks=None, outs=None, sizes=None):
        """The marshalled arguments of one pwrel_compress_batch request over
        FP32 CUDA tensors xs (2-D or 3-D); run() issues the call.  models:
        {ndim: network} for each dimensionality present (use_net); blocks:
        {ndim: block edge} (defaults 16 for 2-D, 8 for 3-D).  outs (one uint8
        tensor per field) and sizes (an int64 tensor of len(xs), each
        stream's length) are allocated when not given.  Running the same
        request again repeats it for the library (same fields, outputs and
        options), which is what a graph capture needs."""
        return BatchRequest(self, xs, eps, models, use_net, judge, independent, blocks, outs,
                            sizes)

    def batch_tiles(self, variants=None):
        """Set (variants = [3-D, 2-D]) and return the batched tile variants and
        their tile extents."""
        if variants is not None:
            v = (C.c_int * 2)(*[int(x) for x in variants])
            self._check(self._L.pwrel_batch_set_tiles(self.h, v), "batch_set_tiles")
        v = (C.c_int * 2)()
        sh = (C.c_int * 6)()
        self._check(self._L.pwrel_batch_get_tiles(self.h, v, sh), "batch_get_tiles")
        return list(v), [tuple(sh[0:3]), tuple(sh[3:6])]

    def compress_batch(self, xs, eps, models=None, use_net=True, judge=False,
                       independent=False, blocks=None, outs=None, sizes=None, stream=None,
                       views=True):
        """One pwrel_compress_batch call (see batch_request).  views=True:
        synchronise and return each field's stream view; else (outs, sizes)
        with the sizes still on the device."""
        r = self.batch_request(xs, eps, models, use_net, judge, independent, blocks, outs,
                               sizes)
        r.run(stream)
        return r.views(stream) if views else (r.outs, r.sizes)

    def openloop(self, x, eps, block=8, model=None, mbits=0, gap=0, stream=None):
        """pwrel_openloop (the paper's literal open-loop prediction, measured):
        returns dict(codes, counts, raw, xhat, report) with device tensors and
        the report as a dict."""
        import torch
        assert x.is_cuda and x.is_contiguous()
        dt = _dtype_code(x.dtype)
        nb = 1
        for s in x.shape:
            nb *= -(-int(s) // int(block))
        codes = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
        counts = torch.empty(nb, dtype=torch.int32, device=x.device)
        raw = torch.empty(max(x.numel(), 1), dtype=x.dtype, device=x.device)
        xh = torch.empty_like(x)
        m = model_struct(model)
        rep = OpenloopReport()
        st = self._L.pwrel_openloop(self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(), dt,
                                    float(eps), int(block), C.byref(m) if m is not None else None,
                                    int(mbits), int(gap), C.c_void_p(codes.data_ptr()),
                                    C.c_void_p(counts.data_ptr()), C.c_void_p(raw.data_ptr()),
                                    raw.numel(), C.c_void_p(xh.data_ptr()), C.byref(rep),
                                    _stream(stream))
        self._check(st, "openloop")
        r = {"n_raw": rep.n_raw, "violations": rep.violations,
             "max_rel_error": rep.max_rel_error, "hist": list(rep.hist), "mbits": rep.mbits,
             "gap": rep.gap}
        return {"codes": codes, "counts": counts, "raw": raw[:rep.n_raw], "xhat": xh,
                "report": r}

    def decompress(self, stream_t, shape=None, dtype=None, out=None, stream=None):
        import torch
        assert stream_t.is_cuda and stream_t.dtype == torch.uint8
        if out is not None:
            # the library checks the output's shape and dtype against the header
            assert out.is_cuda and out.is_contiguous()
            shape = tuple(out.shape) if shape is None else shape
            dtype = out.dtype if dtype is None else dtype
        if shape is None or dtype is None:
            h = header(stream_t)
            shape = tuple(h["dims"][:h["ndim"]])
            dtype = torch.float32 if h["dtype"] == F32 else torch.float64
        if out is None:
            out = torch.empty(shape, dtype=dtype, device=stream_t.device)
        st = self._L.pwrel_decompress(self.h, C.c_void_p(stream_t.data_ptr()), stream_t.numel(),
                                      C.c_void_p(out.data_ptr()), _dims(shape), len(shape),
                                      _dtype_code(dtype), _stream(stream))
        self._check(st, "decompress")
        return out

    def compress_raw(self, x, eps, block=8, model=None, use_net=True, judge=False,
                     independent=False, raw_capacity=None, stream=None):
        """pwrel_compress_raw: the sections of a compression in separate device
        tensors; returns dict(header, codes int16 [n], counts int32 [nblocks],
        bflags uint8 [nblocks] | None, raw [n_raw])."""
        import torch
        assert x.is_cuda and x.is_contiguous()
        dt = _dtype_code(x.dtype)
        n = x.numel()
        nb = 1
        for d in x.shape:
            nb *= -(-int(d) // int(block))
        cap = n if raw_capacity is None else int(raw_capacity)
        codes = torch.empty(max(n, 1), dtype=torch.int16, device=x.device)
        counts = torch.empty(max(nb, 1), dtype=torch.int32, device=x.device)
        bflags = torch.empty(max(nb, 1), dtype=torch.uint8, device=x.device) if judge else None
        raw = torch.empty(max(cap, 1), dtype=x.dtype, device=x.device)
        m = model_struct(model) if use_net else None
        opt = Options(int(bool(use_net)), int(bool(judge)), int(bool(independent)), 0)
        h = Header()
        st = self._L.pwrel_compress_raw(
            self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(), dt, float(eps),
            int(block), C.byref(m) if m is not None else None, C.byref(opt),
            C.c_void_p(codes.data_ptr()), C.c_void_p(counts.data_ptr()),
            C.c_void_p(bflags.data_ptr()) if bflags is not None else None,
            C.c_void_p(raw.data_ptr()), cap, C.byref(h), _stream(stream))
        self._check(st, "compress_raw")
        hd = header_dict(h)
        return {"header": hd, "codes": codes[:n], "counts": counts[:nb],
                "bflags": bflags[:nb] if bflags is not None else None,
                "raw": raw[:hd["n_raw"]]}

    def stream_model(self, stream_t, stream=None):
        """The network stored in a device stream (pwrel_stream_model)."""
        m = Mlp()
        st = self._L.pwrel_stream_model(self.h, C.c_void_p(stream_t.data_ptr()),
                                        stream_t.numel(), C.byref(m), _stream(stream))
        self._check(st, "stream_model")
        return model_dict(m)

    # learned part ------------------------------------------------------------
    def train(self, x, eps, block=8, init=None, rho=0.01, seed=0, hidden=32, alpha=0.01,
              epochs=1, batch=256, lrs=DEFAULT_LRS, lambdas=DEFAULT_LAMBDAS,
              independent=False, precision=1, stream=None):
        """Train a network on the field x (Sec. 4.3); returns (model, report dict)."""
        assert x.is_cuda and x.is_contiguous()
        o = TrainOptions()
        o.rho, o.seed, o.hidden, o.epochs, o.batch = float(rho), int(seed), int(hidden), \
            int(epochs), int(batch)
        o.n_lr, o.n_lambda = len(lrs), len(lambdas)
        for i, v in enumerate(lrs):
            o.lr[i] = float(v)
        for i, v in enumerate(lambdas):
            o.lambda_[i] = float(v)
        o.independent_blocks, o.alpha, o.precision = int(bool(independent)), float(alpha), \
            int(precision)
        m0 = model_struct(init) if init is not None else None
        out = Mlp()
        rep = TrainReport()
        st = self._L.pwrel_train(self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(),
                                 _dtype_code(x.dtype), float(eps), int(block), C.byref(o),
                                 C.byref(m0) if m0 is not None else None, C.byref(out),
                                 C.byref(rep), _stream(stream))
        self._check(st, "train")
        r = {"n_train": rep.n_train, "n_val": rep.n_val, "sigma": rep.sigma,
             "chosen": rep.chosen, "n_candidates": rep.n_candidates,
             "val_score": [rep.val_score[i] for i in range(rep.n_candidates)],
             "ms_sample": rep.ms_sample, "ms_train": rep.ms_train,
             "ms_select": rep.ms_select}
        return model_dict(out), r

    def compress_datablocks(self, x, eps, sub, model=None, use_net=True, judge=False,
                            independent=False, stride=None, stream=None):
        """pwrel_compress_datablocks: a 3-D FP32 field split into data blocks of
        edge `sub`, each its own stream with its own factors (Sec. 5).  Returns
        (streams uint8 [n_sub, stride], sizes uint64 [n_sub]) as CUDA tensors."""
        import torch
        assert x.is_cuda and x.is_contiguous() and x.dim() == 3 and x.dtype == torch.float32
        if stride is None:
            e = max(int(sub), 1)
            stride = compress_bound((min(e, x.shape[0]), min(e, x.shape[1]),
                                     min(e, x.shape[2])), F32, 8)
            stride = (stride + 255) // 256 * 256
        nsub = 1
        for d in x.shape:
            nsub *= -(-int(d) // max(int(sub), 1))  # the library refuses a bad edge
        outs = torch.empty((nsub, stride), dtype=torch.uint8, device=x.device)
        sizes = torch.zeros(nsub, dtype=torch.int64, device=x.device)
        m = model_struct(model) if use_net else None
        opt = Options(int(bool(use_net)), int(bool(judge)), int(bool(independent)), 0)
        n = C.c_uint64(0)
        st = self._L.pwrel_compress_datablocks(
            self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), float(eps), int(sub),
            C.byref(m) if m is not None else None, C.byref(opt), C.c_void_p(outs.data_ptr()),
            int(stride), C.c_void_p(sizes.data_ptr()), C.byref(n), _stream(stream))
        self._check(st, "compress_datablocks")
        assert n.value == nsub
        return outs, sizes

    def decompress_datablocks(self, streams, sizes, shape, sub, out=None, stream=None):
        """pwrel_decompress_datablocks: the field back from compress_datablocks'
        streams ([n_sub, stride] uint8) and sizes (host or device)."""
        import torch
        hs = np.ascontiguousarray(np.asarray(sizes.cpu() if hasattr(sizes, "cpu") else sizes,
                                             dtype=np.uint64))
        if out is None:
            out = torch.empty(tuple(shape), dtype=torch.float32, device=streams.device)
        st = self._L.pwrel_decompress_datablocks(
            self.h, C.c_void_p(streams.data_ptr()), int(streams.shape[1]),
            hs.ctypes.data_as(_P), C.c_void_p(out.data_ptr()), _dims(shape), int(sub),
            _stream(stream))
        self._check(st, "decompress_datablocks")
        return out

    def train_codebook(self, x, eps, block=8, model=None, use_net=True, judge=False,
                       independent=False, frac=0.02, seed=0, stream=None):
        """The Huffman table of the training phase (Sec. 4.3): the field
        compressed with these options, the code counts of its validation
        blocks (a `frac` share, drawn with `seed`), one table from them; a
        Codebook for compress(codebook=...)."""
        assert x.is_cuda and x.is_contiguous()
        m = model_struct(model) if use_net else None
        opt = Options(int(bool(use_net)), int(bool(judge)), int(bool(independent)), 0)
        cb = Codebook()
        st = self._L.pwrel_train_codebook(self.h, C.c_void_p(x.data_ptr()), _dims(x.shape),
                                          x.dim(), _dtype_code(x.dtype), float(eps), int(block),
                                          C.byref(m) if m is not None else None, C.byref(opt),
                                          float(frac), int(seed), C.byref(cb), _stream(stream))
        self._check(st, "train_codebook")
        return cb

    def sample(self, x, eps, block=8, independent=False, rho=0.01, seed=0, stream=None):
        """Training/validation pairs of x in ascending point order:
        (idx uint64, u int32 [n, K], t int32, isval uint8) as CUDA tensors."""
        import torch
        K = (1 << x.dim()) - 2
        n = C.c_uint64(0)
        args = (self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(), _dtype_code(x.dtype),
                float(eps), int(block), int(bool(independent)), float(rho), int(seed))
        st = self._L.pwrel_sample(*args, None, None, None, None, 0, C.byref(n),
                                  _stream(stream))
        self._check(st, "sample")
        cnt = n.value
        dev = x.device
        idx = torch.empty(max(cnt, 1), dtype=torch.int64, device=dev)
        u = torch.empty((max(cnt, 1), max(K, 1)), dtype=torch.int32, device=dev)
        t = torch.empty(max(cnt, 1), dtype=torch.int32, device=dev)
        iv = torch.empty(max(cnt, 1), dtype=torch.uint8, device=dev)
        st = self._L.pwrel_sample(*args, C.c_void_p(idx.data_ptr()), C.c_void_p(u.data_ptr()),
                                  C.c_void_p(t.data_ptr()), C.c_void_p(iv.data_ptr()), cnt,
                                  C.byref(n), _stream(stream))
        self._check(st, "sample")
        return idx[:cnt], u[:cnt, :K], t[:cnt], iv[:cnt]

    def loss_grad(self, theta, hidden, inputs, alpha, u, t, sigma, lam, stream=None):
        """Loss and gradient (FP32) of scaled-domain parameters on pairs (u, t)."""
        import torch
        theta = theta.contiguous()
        g = torch.empty_like(theta)
        loss = C.c_float(0.0)
        st = self._L.pwrel_loss_grad(self.h, C.c_void_p(theta.data_ptr()), int(hidden),
                                     int(inputs), float(alpha), C.c_void_p(u.data_ptr()),
                                     C.c_void_p(t.data_ptr()), t.numel(), float(sigma),
                                     float(lam), C.c_void_p(g.data_ptr()), C.byref(loss),
                                     _stream(stream))
        self._check(st, "loss_grad")
        return float(loss.value), g

    def train_pairs(self, u, t, hidden, inputs, alpha, sigma, theta0, lrs, lambdas, batch=256,
                    epochs=1, stream=None):
        """Adam-train len(lrs) candidates from theta0 on pairs; returns [n_cand, P]."""
        import torch
        nc = len(lrs)
        P = hidden * inputs + 2 * hidden + 1
        out = torch.empty((nc, P), dtype=torch.float32, device=t.device)
        lr = (C.c_double * nc)(*[float(v) for v in lrs])
        lm = (C.c_double * nc)(*[float(v) for v in lambdas])
        st = self._L.pwrel_train_pairs(self.h, C.c_void_p(u.data_ptr()), C.c_void_p(t.data_ptr()),
                                       t.numel(), int(hidden), int(inputs), float(alpha),
                                       float(sigma), C.c_void_p(theta0.data_ptr()), nc,
                                       C.cast(lr, _P), C.cast(lm, _P), int(batch), int(epochs),
                                       C.c_void_p(out.data_ptr()), _stream(stream))
        self._check(st, "train_pairs")
        return out

    # inspection ----------------------------------------------------------------
    def transform(self, x, eps, stream=None):
        import torch
        p = torch.empty(x.shape, dtype=torch.int32, device=x.device)
        h = Header()
        st = self._L.pwrel_transform(self.h, C.c_void_p(x.data_ptr()), _dims(x.shape), x.dim(),
                                     _dtype_code(x.dtype), float(eps), C.c_void_p(p.data_ptr()),
                                     C.byref(h), _stream(stream))
        self._check(st, "transform")
        return p, header_dict(h)

    def encode_grid(self, p, block, model=None, use_net=True, independent=False, stream=None):
        import torch
        assert p.dtype == torch.int32 and p.is_cuda and p.is_contiguous()
        codes = torch.empty(p.numel(), dtype=torch.int16, device=p.device)
        m = model_struct(model) if use_net else None
        opt = Options(int(bool(use_net)), 0, int(bool(independent)), 0)
        st = self._L.pwrel_encode_grid(self.h, C.c_void_p(p.data_ptr()), _dims(p.shape), p.dim(),
                                       int(block), C.byref(m) if m is not None else None,
                                       C.byref(opt), C.c_void_p(codes.data_ptr()),
                                       _stream(stream))
        self._check(st, "encode_grid")
        return codes

    def detmath(self, x, stream=None):
        import torch
        assert x.dtype == torch.float64 and x.is_cuda
        l2 = torch.empty_like(x)
        e2 = torch.empty_like(x)
        st = self._L.pwrel_detmath(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(l2.data_ptr()),
                                   C.c_void_p(e2.data_ptr()), x.numel(), _stream(stream))
        self._check(st, "detmath")
        return l2, e2

    def fastmath_check(self, stream=None):
        """Largest errors of the FP32 fast-path log2 / exp2 over every input
        they can receive: (log2 absolute error, exp2 relative error)."""
        a, b = C.c_double(0.0), C.c_double(0.0)
        self._check(self._L.pwrel_fastmath_check(self.h, C.byref(a), C.byref(b),
                                                 _stream(stream)), "fastmath_check")
        return a.value, b.value

    def set_profiling(self, enable=True):
        self._check(self._L.pwrel_set_profiling(self.h, int(bool(enable))), "set_profiling")

    def phase_times(self):
        ms = (C.c_double * len(PHASES))()
        n = self._L.pwrel_phase_times(self.h, C.cast(ms, _P), len(PHASES))
        return {PHASES[i]: ms[i] for i in range(n)}

    def histogram(self, codes, stream=None):
        """65536-bin histogram of a device tensor of codes (int16 / uint16 view)."""
        hist = np.zeros(65536, dtype=np.uint64)
        st = self._L.pwrel_histogram(self.h, C.c_void_p(codes.data_ptr()), codes.numel(),
                                     hist.ctypes.data_as(_P), _stream(stream))
        self._check(st, "histogram")
        return hist


# --- stream inspection (host copies of the sections) ------------------------------

class BatchRequest:
    """Arguments of pwrel_compress_batch built once (field table, models,
    options, outputs); run() passes them to the library."""

    def __init__(self, ctx, xs, eps, models, use_net, judge, independent, blocks, outs, sizes):
        import torch
        n = len(xs)
        self.ctx, self.xs, self.eps = ctx, list(xs), float(eps)
        blocks = dict(blocks or {})
        self.bs = (C.c_int * 3)(0, int(blocks.get(2, 16)), int(blocks.get(3, 8)))
        if outs is None:
            outs = []
            for x in xs:
                cap = compress_bound(x.shape, _dtype_code(x.dtype), self.bs[x.dim() - 1])
                outs.append(torch.empty(max(cap, 1), dtype=torch.uint8, device=x.device))
        if sizes is None:
            sizes = torch.zeros(n, dtype=torch.int64, device=xs[0].device)
        self.outs, self.sizes = list(outs), sizes
        self.descs = (FieldDesc * n)()
        for i, (x, o) in enumerate(zip(xs, outs)):
            assert x.is_cuda and x.is_contiguous()
            d = self.descs[i]
            d.d_field = x.data_ptr()
            for k, s in enumerate(x.shape):
                d.dims[k] = int(s)
            d.ndim = x.dim()
            d.d_out = o.data_ptr()
            d.out_capacity = o.numel()
        self.keep = {}
        self.mptrs = (C.POINTER(Mlp) * 3)()
        if use_net:
            for nd, m in (models or {}).items():
                self.keep[nd] = model_struct(m)
                self.mptrs[nd - 1] = C.pointer(self.keep[nd])
        self.opt = Options(int(bool(use_net)), int(bool(judge)), int(bool(independent)), 0)
        self.dt = _dtype_code(xs[0].dtype) if n else F32

    def tune(self, reps=3, stream=None):
        """pwrel_compress_batch_tune over this request: returns (variants
        [3-D, 2-D], median ms [class][variant]); the context keeps them."""
        c = self.ctx
        var = (C.c_int * 2)()
        ms = (C.c_double * (2 * BATCH_TILES))()
        st = c._L.pwrel_compress_batch_tune(c.h, len(self.xs), self.descs, self.dt, self.eps,
                                            C.cast(self.bs, C.c_void_p), self.mptrs,
                                            C.byref(self.opt), C.c_void_p(self.sizes.data_ptr()),
                                            int(reps), var, ms, _stream(stream))
        c._check(st, "compress_batch_tune")
        return list(var), [list(ms[k * BATCH_TILES:(k + 1) * BATCH_TILES]) for k in range(2)]

    def run(self, stream=None):
        c = self.ctx
        st = c._L.pwrel_compress_batch(c.h, len(self.xs), self.descs, self.dt, self.eps,
                                       C.cast(self.bs, C.c_void_p), self.mptrs,
                                       C.byref(self.opt), C.c_void_p(self.sizes.data_ptr()),
                                       _stream(stream))
        c._check(st, "compress_batch")

    def views(self, stream=None):
        """Synchronise `stream` and return each field's stream (empty where
        the field failed)."""
        import torch
        if stream is not None:
            stream.synchronize()
        else:
            torch.cuda.current_stream(self.sizes.device).synchronize()
        return [o[:s] for o, s in zip(self.outs, self.sizes.cpu().tolist())]


def header(stream_t):
    """Parse and validate the header of a device stream tensor."""
    head = stream_t[:HEADER_BYTES].cpu().numpy().tobytes()
    return read_header_bytes(head, size=stream_t.numel())


def sections(stream_t):
    """Header dict plus the sections of a device stream, as device tensor views
    (only the header and the model are copied to the host)."""
    import torch
    head = stream_t[:HEADER_BYTES + C.sizeof(Mlp)].cpu().numpy().tobytes()
    h = read_header_bytes(head, size=stream_t.numel())
    raw = head
    n, nb, nr = h["n"], h["nblocks"], h["n_raw"]
    tdt = torch.float32 if h["dtype"] == F32 else torch.float64
    tsz = 4 if h["dtype"] == F32 else 8

    def view(off, count, dt, size):
        return stream_t[off:off + count * size].view(dt)

    out = {"header": h,
           "counts": view(h["off_counts"], nb, torch.int32, 4),
           "raw": view(h["off_raw"], nr, tdt, tsz)}
    if h["flags"] & HF_HUFFMAN:
        # codebook: counts of each length, symbols in canonical order; per-block
        # bit sizes; the packed words
        out["huff_count"] = view(h["off_huff"], HUFF_MAX_LEN + 1, torch.int32, 4)
        out["huff_syms"] = view(h["off_huff"] + 4 * (HUFF_MAX_LEN + 1), h["n_sym"],
                                torch.int16, 2)
        out["sizes"] = view(h["off_sizes"], nb, torch.int16 if h["size_bytes"] == 2
                            else torch.int32, h["size_bytes"])
        out["bits"] = view(h["off_bits"], (h["n_bits"] + 31) // 32, torch.int32, 4)
    else:
        out["codes"] = view(h["off_codes"], n, torch.int16, 2)
    if h["flags"] & HF_JUDGE:
        out["bflags"] = stream_t[h["off_bflags"]:h["off_bflags"] + nb]
    if h["flags"] & HF_NET:
        m = Mlp.from_buffer_copy(raw[h["off_model"]:h["off_model"] + C.sizeof(Mlp)])
        out["model"] = model_dict(m)
    return out
