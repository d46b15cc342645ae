"""The oracle's open-loop mode (the paper's literal data selection: predict
from the neighbours' raw log-domain values; Sec. 4.3, 4.4.1, 4.4.2) pinned
on the CPU: against the independent brute force on tiny fields (codes,
counts, raw values, the coverage histogram, the decoded field and its
coordinates, bit for bit), against closed forms (1-D Lorenzo decoding is a
running sum of rounded differences; a point predicted only from balance
points errs by at most half a grid step), and against the special cases
(every point a balance point reproduces the field; the coordinate of an
integer grid value inverts like the grid value)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as BF


def _field(shape, seed, dtype=np.float32, neg=0.15, zero=0.05):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    base = np.cumsum(rng.standard_normal(n)).reshape(shape) * 0.2
    x = np.exp(base) * np.where(rng.random(shape) < neg, -1.0, 1.0)
    x = x.astype(dtype)
    x.reshape(-1)[rng.random(n) < zero] = 0
    return x


def _model(ndim, H, seed):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, 0.2, size=(H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 0.5, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.2, H)).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal(0, 0.3)))
    return m


BF_CASES = [
    ("1d", (23,), 4, None, 16, 0),
    ("1d_m4_gap3", (23,), 5, None, 4, 3),
    ("2d", (7, 9), 4, None, 16, 0),
    ("2d_net", (7, 9), 4, (2, 4, 3), 16, 0),
    ("2d_m3", (6, 7), 3, None, 3, 0),
    ("3d", (4, 5, 6), 3, None, 16, 0),
    ("3d_net_gap", (4, 5, 6), 3, (3, 4, 5), 8, 4),
    ("3d_f64", (5, 4, 3), 2, None, 6, 2),
]


@pytest.mark.parametrize("name,shape,B,net,mbits,gap", BF_CASES, ids=[c[0] for c in BF_CASES])
def test_openloop_matches_bruteforce(name, shape, B, net, mbits, gap):
    dtype = np.float64 if name.endswith("f64") else np.float32
    x = _field(shape, hash(name) % 1000, dtype)
    model = _model(*net) if net else None
    eps = 1e-2
    r = O.openloop_encode(x, eps, B, model, mbits, gap)
    codes, counts, raw, hist, c = BF.ol_compress(x, eps, B, model, mbits, gap)
    assert r["codes"].tolist() == codes
    assert r["counts"].tolist() == counts
    assert np.array_equal(r["raw"].astype(np.float64), np.array(raw, dtype=np.float64))
    assert r["hist"].tolist() == hist
    for k in ("w", "Lp", "Ln", "p_zero", "b_sign", "delta"):
        assert r["consts"][k] == c[k], k
    xh, t = O.openloop_decode(r["codes"], r["raw"], r["consts"], shape, dtype, B, model, mbits)
    bxh, bt = BF.ol_decompress(codes, raw, c, shape, dtype == np.float32, B, model, mbits)
    for coord, v in bxh.items():
        assert xh[coord] == v or (math.isnan(v) and np.isnan(xh[coord])), coord
        assert t[coord] == bt[coord], coord


def test_every_point_a_balance_point_reproduces_the_field():
    x = _field((9, 10, 11), 5)
    r = O.openloop_encode(x, 1e-2, 4, None, 16, gap=1)
    assert np.all(r["codes"] == 0) and r["raw"].size == x.size
    xh, _ = O.openloop_decode(r["codes"], r["raw"], r["consts"], x.shape, x.dtype, 4, None, 16)
    assert np.array_equal(xh.view(np.uint32), x.view(np.uint32))


def test_1d_lorenzo_decoding_is_a_running_sum_of_rounded_differences():
    """1-D Lorenzo: the decoder's coordinate is the block's first value plus
    the rounded raw differences, t^_i = t_0 + sum_{j<=i} rint(t_j - t_{j-1})."""
    x = _field((200,), 11, neg=0.0, zero=0.0)
    B = 64
    r = O.openloop_encode(x, 1e-3, B, None, 16, 0)
    c = r["consts"]
    t = O.tcoord(x, c)
    assert np.all(r["counts"] == 1)  # only the blocks' first points are balance points
    _, th = O.openloop_decode(r["codes"], r["raw"], c, x.shape, x.dtype, B, None, 16)
    for b0 in range(0, 200, B):
        acc = float(t[b0])
        assert th[b0] == acc
        for i in range(b0 + 1, min(b0 + B, 200)):
            acc = acc + float(np.rint(t[i] - t[i - 1]))
            assert th[i] == acc, i
            assert r["codes"][i] == int(np.rint(t[i - 1] - t[i])) + 32768


def test_points_predicted_from_balance_points_err_by_half_a_step():
    """Second point of each 1-D block: its only neighbour is the block's exact
    first point, so the decoder's prediction equals the encoder's."""
    x = _field((90,), 12, neg=0.2, zero=0.0)
    B = 10
    r = O.openloop_encode(x, 1e-2, B, None, 16, 0)
    t = O.tcoord(x, r["consts"])
    _, th = O.openloop_decode(r["codes"], r["raw"], r["consts"], x.shape, x.dtype, B, None, 16)
    for i in range(1, 90, B):
        assert abs(th[i] - t[i]) <= 0.5


def test_integer_coordinate_inverts_like_the_grid_value():
    x = _field((500,), 13)
    c = O.consts(x, 1e-2)
    p = O.transform_field(x, c).ravel()
    t = O.tcoord(x, c).ravel()
    # rounding the coordinate gives the grid value wherever no clamp applies
    agree = np.rint(t) == p
    assert agree.mean() > 0.99
    xi = O.tinverse(p.astype(np.float64), c, np.float32)
    assert np.array_equal(xi.view(np.uint32), O.inverse_field(p, c, np.float32).ravel().view(np.uint32))


def test_coverage_choice():
    hist = np.zeros(18, np.uint64)
    # coverage by m = 1 .. 5: 10, 20, 40, 65, 90 of 100 points (10 never covered)
    hist[[1, 2, 3, 4, 5, 17]] = [10, 10, 20, 25, 25, 10]
    assert O.openloop_choose_m(hist, 1e-2) == 3    # below 1.5%: closest to 50% is 40%
    assert O.openloop_choose_m(hist, 2e-2) == 5    # from 1.5%: closest to 80% is 90%
    assert O.openloop_choose_m(hist, 1.5e-2) == 5
    even = np.zeros(18, np.uint64)
    even[[2, 3, 17]] = [50, 50, 100]                # 25% and 50%: m = 3 hits 50% exactly
    assert O.openloop_choose_m(even, 1e-3) == 3


def test_drift_breaks_the_bound_where_the_grid_snapped_reading_does_not():
    """The reason for the grid-snapped reading: on a rough 3-D field the
    open-loop decoder violates the bound; the closed-loop codec never does."""
    x = _field((16, 16, 16), 14)
    r = O.openloop_encode(x, 1e-2, 8, None, 16, 0)
    xh, _ = O.openloop_decode(r["codes"], r["raw"], r["consts"], x.shape, x.dtype, 8, None, 16)
    assert O.openloop_report(x, xh, 1e-2)["violations"] > 0
    ref = O.compress(x, 1e-2, 8, None, O.MODE_LORENZO, independent=True)
    xc, _ = O.decompress(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, 8, None,
                         O.MODE_LORENZO, independent=True)
    assert O.openloop_report(x, xc, 1e-2)["violations"] == 0
