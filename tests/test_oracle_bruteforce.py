"""The C oracle against the independent brute-force implementation on tiny
random fields: codes, per-block counts, raw lists, constants and the decoded
field must agree bit for bit (CPU only)."""
import zlib

import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as BF


def _field(shape, seed, dtype, kind):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    if kind == "smooth":
        base = np.cumsum(rng.standard_normal(n)).reshape(shape) * 0.05
        x = np.exp(base) * np.where(rng.random(shape) < 0.15, -1.0, 1.0)
    elif kind == "wild":
        x = rng.standard_normal(shape) * 10.0 ** rng.uniform(-6, 6, shape)
    else:  # "tiny": subnormals and zeros
        lo = -40 if dtype == np.float32 else -310
        x = rng.standard_normal(shape) * 10.0 ** rng.uniform(lo, lo + 8, shape)
    x = x.astype(dtype)
    x.reshape(-1)[rng.random(n) < 0.08] = 0
    return x


def _random_model(ndim, H, seed):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, 0.2, size=(H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 0.5, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.2, H)).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal(0, 0.3)))
    return m


CASES = [
    ((6, 5, 7), 4, np.float32, "smooth", 1e-2, False),
    ((5, 6, 6), 3, np.float32, "wild", 1e-3, False),
    ((6, 6, 5), 4, np.float64, "wild", 1e-4, True),
    ((4, 5, 6), 2, np.float32, "tiny", 1e-1, False),
    ((4, 4, 7), 4, np.float64, "tiny", 1e-2, True),
    ((11, 13), 4, np.float32, "smooth", 1e-2, False),
    ((9, 14), 5, np.float64, "wild", 1e-3, True),
    ((40,), 8, np.float32, "wild", 1e-2, False),
    ((33,), 4, np.float64, "smooth", 1e-3, True),
]


@pytest.mark.parametrize("shape,B,dtype,kind,eps,indep", CASES)
@pytest.mark.parametrize("net", ["lorenzo", "init", "random"])
def test_oracle_equals_bruteforce(shape, B, dtype, kind, eps, indep, net):
    D = len(shape)
    seed = zlib.crc32(repr((shape, B, kind, net)).encode()) % 1000
    x = _field(shape, seed, dtype, kind)
    if net == "lorenzo":
        model, mode = None, O.MODE_LORENZO
    elif net == "init":
        model, mode = O.mlp_init(D, 4, seed=5) if D > 1 else O.mlp_init(1, 2), O.MODE_PLAIN
    else:
        model, mode = _random_model(D, 5, seed), O.MODE_PLAIN
    ora = O.compress(x, eps, B, model, mode, independent=indep)
    codes, counts, raw, c, P = BF.compress(x, eps, B, model, indep)
    for k in ("eps0", "b_a", "w", "r", "Lp", "Ln", "d0", "p_zero", "b_sign", "n_lo", "delta"):
        assert ora["consts"][k] == c[k], k
    assert ora["codes"].tolist() == codes
    assert ora["counts"].tolist() == counts
    assert [float(v) for v in ora["raw"]] == raw
    xh_o, p_o = O.decompress(ora["codes"], ora["raw"], ora["consts"], shape, dtype, B, model,
                             mode, independent=indep)
    xh_b, P_b = BF.decompress(codes, raw, c, shape, dtype == np.float32, B, model, indep)
    for coord, v in xh_b.items():
        assert float(xh_o[coord]) == v or (np.isnan(v) and np.isnan(xh_o[coord]))
        assert p_o[coord] == P_b[coord]
