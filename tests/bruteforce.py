"""Independent brute-force implementation of the compressor for tiny fields.

Written separately from the C oracle (no shared code, a different control
structure): every point is handled through Python dictionaries keyed by
coordinates, the stream order comes from sorting points by (block raster key,
local raster key), every fused multiply-add is evaluated exactly with
fractions.Fraction and rounded once, and FP32 rounding is done by hand.
Only meant for fields of a few hundred points.
"""
from fractions import Fraction
import itertools
import math
import struct

R = 32768


# --- exact rounding -------------------------------------------------------------

def round_binary(q, mant_bits, emin, emax):
    """Round a Fraction to the nearest binary floating-point number with
    `mant_bits` significand bits (ties to even), subnormals below 2^emin,
    overflow to +-inf above the largest finite value."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    if Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    scale = e - (mant_bits - 1)
    m = a / (Fraction(2) ** scale)
    n = m.numerator // m.denominator
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    val = Fraction(n) * Fraction(2) ** scale
    maxv = (2 - Fraction(2) ** (1 - mant_bits)) * Fraction(2) ** emax
    if val > maxv:
        return sign * math.inf
    return sign * float(val)


def f32(q):
    return round_binary(Fraction(q), 24, -126, 127)


def f64(q):
    return round_binary(Fraction(q), 53, -1022, 1023)


def fma64(a, b, c):
    return f64(Fraction(a) * Fraction(b) + Fraction(c))


def fma32(a, b, c):
    return f32(Fraction(a) * Fraction(b) + Fraction(c))


def mul32(a, b):
    return f32(Fraction(a) * Fraction(b))


# --- deterministic log2 / exp2 (same published series, own code) ---------------

def det_log2(x):
    assert x > 0 and math.isfinite(x)
    eadj = 0
    if x < 2.0 ** -1022:
        x = x * 2.0 ** 54
        eadj = -54
    m, e = math.frexp(x)          # x = m 2^e, m in [0.5, 1)
    m, e = m * 2.0, e - 1         # m in [1, 2)
    if m > 1.4142135623730951:
        m, e = m * 0.5, e + 1
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    coef = [1.0 / (2 * k + 1) for k in range(11)]
    P = coef[10]
    for k in range(9, -1, -1):
        P = fma64(P, z, coef[k])
    return float(e + eadj) + ((s + s) * P) * 1.4426950408889634


def det_exp2(t):
    k = round(t)                  # ties to even, like rint
    f = t - k
    a = f * 0.6931471805599453
    coef = [1.0 / math.factorial(j) for j in range(14)]
    P = coef[13]
    for j in range(12, -1, -1):
        P = fma64(P, a, coef[j])
    return f64(Fraction(P) * Fraction(2) ** int(k))


# --- constants and point maps ---------------------------------------------------

def constants(values, is_f32, eps):
    nz = [abs(v) for v in values if v != 0.0]
    amin, amax = (min(nz), max(nz)) if nz else (1.0, 1.0)
    tau = 2.0 ** -126 if is_f32 else 2.0 ** -1022
    eps0 = min(tau, amin * 0.5)
    b_a = det_log2(1.0 + eps)
    w = b_a + b_a
    r = 1.0 / w
    Lp = det_log2(amin)
    Ln = ((det_log2(amax + eps0) + Lp) + w) - det_log2(amin - eps0)
    d0 = det_log2(eps0) + Lp
    p_zero = round(d0 * r)
    b_sign = round((det_log2(amax) + Lp) * r)
    n_lo = round((det_log2(amin) + Ln) * r)
    delta = max(0, b_sign + 1 - n_lo)
    return dict(eps=eps, eps0=eps0, b_a=b_a, w=w, r=r, Lp=Lp, Ln=Ln, d0=d0, p_zero=p_zero,
                b_sign=b_sign, n_lo=n_lo, delta=delta)


def to_grid(x, c):
    if x == 0.0:
        return c["p_zero"]
    if x > 0:
        q = round((det_log2(x) + c["Lp"]) * c["r"])
        return min(max(q, c["p_zero"] + 1), c["b_sign"])
    q = round((det_log2(-x) + c["Ln"]) * c["r"]) + c["delta"]
    return max(q, c["b_sign"] + 1)


def from_grid(p, c, is_f32):
    if p <= c["p_zero"]:
        v = 0.0
    elif p <= c["b_sign"]:
        v = det_exp2(float(p) * c["w"] - c["Lp"])
    else:
        v = -det_exp2(float(p - c["delta"]) * c["w"] - c["Ln"])
    return f32(v) if (is_f32 and math.isfinite(v)) else v


def within_bound(x, xh, eps):
    if x == 0.0:
        return xh == 0.0
    if xh == 0.0 or (x < 0) != (xh < 0):
        return False
    return abs(x - xh) <= eps * abs(x)


# --- prediction -------------------------------------------------------------------

def offsets(D):
    """(o, coordinate step) for o = 1 .. 2^D - 1; bit i of o = axis D-1-i."""
    out = []
    for o in range(1, 1 << D):
        step = tuple((o >> (D - 1 - d)) & 1 for d in range(D))
        out.append((o, step))
    return out


def lorenzo_sign(step):
    return 1 if sum(step) % 2 == 1 else -1


def net_value(model, u):
    """FP32 network value with exact single-rounding fma (Sec. 4.2)."""
    H = len(model["b1"])
    alpha = float(model["alpha"])
    h = []
    for j in range(H):
        z = float(model["b1"][j])
        for k, uk in enumerate(u):
            z = fma32(float(model["w1"][j][k]), uk, z)
        h.append(mul32(z, alpha) if z < 0 else z)
    y = float(model["b2"])
    for j in range(H):
        y = fma32(float(model["v"][j]), h[j], y)
    return y


def predict(P, coord, shape, B, independent, model):
    D = len(shape)
    nbr = {}
    for o, step in offsets(D):
        q = tuple(a - s for a, s in zip(coord, step))
        ok = all(v >= 0 for v in q)
        if ok and independent:
            ok = all(a // B == b // B for a, b in zip(q, coord))
        if ok:
            nbr[o] = P[q]
    if model is not None and len(nbr) == (1 << D) - 1:
        u = [f32(nbr[k + 2] - nbr[1]) for k in range((1 << D) - 2)]
        y = net_value(model, u)
        y = min(y, 2.0 ** 30)
        y = max(y, -(2.0 ** 30))
        return nbr[1] + round(y)
    return sum(lorenzo_sign(step) * nbr[o] for o, step in offsets(D) if o in nbr)


# --- stream order -------------------------------------------------------------------

def stream_order(shape, B):
    """All coordinates sorted by (block raster key, local raster key)."""
    pts = list(itertools.product(*[range(n) for n in shape]))
    return sorted(pts, key=lambda c: (tuple(v // B for v in c), tuple(v % B for v in c)))


def block_index(coord, shape, B):
    nb = [-(-n // B) for n in shape]
    i = 0
    for v, m in zip(coord, nb):
        i = i * m + v // B
    return i


# --- whole codec --------------------------------------------------------------------

def compress(x, eps, B, model=None, independent=False):
    """x: numpy array (float32 or float64).  Returns codes, counts, raw, consts, P."""
    shape = x.shape
    is_f32 = x.dtype.itemsize == 4
    vals = {c: float(x[c]) for c in itertools.product(*[range(n) for n in shape])}
    c = constants(list(vals.values()), is_f32, eps)
    P = {k: to_grid(v, c) for k, v in vals.items()}
    nb = 1
    for n in shape:
        nb *= -(-n // B)
    counts = [0] * nb
    codes, raw = [], []
    for coord in stream_order(shape, B):
        pred = predict(P, coord, shape, B, independent, model)
        xv = vals[coord]
        ok = within_bound(xv, from_grid(P[coord], c, is_f32), eps)
        e = pred - P[coord]
        if ok and -R < e < R:
            codes.append(e + R)
        else:
            codes.append(0)
            raw.append(xv)
            counts[block_index(coord, shape, B)] += 1
    return codes, counts, raw, c, P


def decompress(codes, raw, c, shape, is_f32, B, model=None, independent=False):
    P, xh = {}, {}
    it = iter(raw)
    for code, coord in zip(codes, stream_order(shape, B)):
        if code:
            P[coord] = predict(P, coord, shape, B, independent, model) - (code - R)
            xh[coord] = from_grid(P[coord], c, is_f32)
        else:
            v = next(it)
            xh[coord] = v
            P[coord] = to_grid(v, c)
    return xh, P


def f32_bits(v):
    return struct.unpack("<I", struct.pack("<f", v))[0]


# --- open-loop mode (raw-coordinate prediction, drifting decoder) ----------------------

def ol_coord(x, c):
    """Continuous grid coordinate (before rounding)."""
    if x == 0.0:
        return float(c["p_zero"])
    if x > 0:
        return (det_log2(x) + c["Lp"]) * c["r"]
    return (det_log2(-x) + c["Ln"]) * c["r"] + float(c["delta"])


def ol_inverse(t, c, is_f32):
    q = round(t)
    if q <= c["p_zero"]:
        v = 0.0
    elif q <= c["b_sign"]:
        v = det_exp2(t * c["w"] - c["Lp"])
    else:
        v = -det_exp2((t - float(c["delta"])) * c["w"] - c["Ln"])
    return f32(v) if (is_f32 and math.isfinite(v)) else v


def ol_predict(T, coord, shape, B, model):
    D = len(shape)
    nbr = {}
    for o, step in offsets(D):
        q = tuple(a - s for a, s in zip(coord, step))
        if all(v >= 0 for v in q) and all(a // B == b // B for a, b in zip(q, coord)):
            nbr[o] = T[q]
    if model is not None and len(nbr) == (1 << D) - 1:
        u = [f32(nbr[k + 2] - nbr[1]) for k in range((1 << D) - 2)]
        return nbr[1] + net_value(model, u)
    s = 0.0
    for o, step in offsets(D):
        if o in nbr:
            s = s + nbr[o] if lorenzo_sign(step) > 0 else s - nbr[o]
    return s


def ol_compress(x, eps, B, model=None, mbits=16, gap=0):
    """Returns codes, counts, raw, hist (hist[m] = errors first fitting m bits), consts."""
    shape = x.shape
    is_f32 = x.dtype.itemsize == 4
    vals = {k: float(x[k]) for k in itertools.product(*[range(n) for n in shape])}
    c = constants(list(vals.values()), is_f32, eps)
    T = {k: ol_coord(v, c) for k, v in vals.items()}
    half = 2 ** (mbits - 1)
    nb = 1
    for n in shape:
        nb *= -(-n // B)
    counts, codes, raw, hist = [0] * nb, [], [], [0] * 18
    last_block, since = None, 0
    for coord in stream_order(shape, B):
        b = block_index(coord, shape, B)
        cq = round(ol_predict(T, coord, shape, B, model) - T[coord])
        need = next((m for m in range(1, 17) if abs(cq) < 2 ** (m - 1)), 17)
        hist[need] += 1
        first = b != last_block
        last_block = b
        balance = first or not abs(cq) < half
        if not balance and gap > 0 and since + 1 >= gap:
            balance = True
        since = 0 if balance else since + 1
        if balance:
            codes.append(0)
            raw.append(vals[coord])
            counts[b] += 1
        else:
            codes.append(cq + half)
    return codes, counts, raw, hist, c


def ol_decompress(codes, raw, c, shape, is_f32, B, model=None, mbits=16):
    half = 2 ** (mbits - 1)
    T, xh = {}, {}
    it = iter(raw)
    for code, coord in zip(codes, stream_order(shape, B)):
        if code:
            T[coord] = ol_predict(T, coord, shape, B, model) - float(code - half)
            xh[coord] = ol_inverse(T[coord], c, is_f32)
        else:
            v = next(it)
            xh[coord] = v
            T[coord] = ol_coord(v, c)
    return xh, T
