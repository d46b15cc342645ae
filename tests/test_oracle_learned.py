"""Pins of the oracle's learned-path pieces (Sec. 4.2 / 4.3), CPU only.

- per-block judge score: closed forms (a constant block has zero entropy, a
  block of distinct codes has J = 0), every distinct code is a symbol of its
  own however large its error (no clamping), the balance point is a symbol of
  its own, and n q(n) - J against an entropy computed here with numpy over
  the full multiset of codes;
- the judge inside the oracle's compressor (mode 2): each block's flag is the
  comparison of the two scores of that block, and the block carries the codes
  of the predictor that won;
- the BF16 error bound: it covers the oracle's BF16 reference and a second
  admissible BF16 evaluation written here (unsplit leaky ReLU, another
  summation order); it is tight where the roundings of a hand-built network
  line up; it is zero-width where every operand is a bf16 number;
- the BF16 reference network (a secondary check): hand-computed values for
  networks whose operands are (or are not) bfloat16-representable, and the
  Lorenzo-equivalent network reproducing Lorenzo exactly where every operand
  is representable.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2309_09778_amd import synth

R = 32768
Q1 = 2 ** 32  # q(2) = rint(2^32 log2 2)


def test_judge_closed_forms():
    for code in (0, R, R + 5, R - 900):
        for n in (1, 2, 7, 512):
            assert O.judge_j(np.full(n, code)) == n * O.qlog(n)
    # distinct bins: every count is 1, q(1) = 0
    assert O.judge_j(np.array([0, R, R + 1, R - 1, R + 127, R - 127])) == 0
    assert O.qlog(1) == 0 and O.qlog(2) == Q1 and O.qlog(4) == 2 * Q1


def test_judge_counts_every_code_as_its_own_symbol():
    # large errors are distinct symbols, not one end bin
    assert O.judge_j(np.array([R + 200, R + 127])) == 0
    assert O.judge_j(np.array([R - 300, R - 127, R - 32767])) == 0
    assert O.judge_j(np.array([R + 200, R + 200, R + 201])) == 2 * Q1
    assert O.judge_j(np.array([1, 1, 65535, 65535])) == 2 * 2 * Q1
    # code 0 (balance point) is not error 0
    assert O.judge_j(np.array([0, R])) == 0
    assert O.judge_j(np.array([R, R])) == 2 * Q1
    assert O.judge_j(np.array([0, 0, R])) == 2 * Q1


def test_judge_order_free_and_large_errors_decide():
    # 512 distinct large errors (9 bits each) lose to two symbols within a
    # narrow range (1 bit each); a score that lumped the large errors into
    # one bin would pick the other way
    wide = (R + 128 + np.arange(512)).astype(np.uint16)
    two = np.where(np.arange(512) % 2 == 0, R + 3, R - 3).astype(np.uint16)
    assert O.judge_j(wide) == 0
    assert O.judge_j(two) == 512 * O.qlog(256) == 512 * 8 * Q1
    assert O.judge_j(two) > O.judge_j(wide)
    rng = np.random.default_rng(1)
    c = rng.integers(0, 65536, 777).astype(np.uint16)
    c[::3] = c[1]
    assert O.judge_j(c) == O.judge_j(rng.permutation(c))


def test_judge_score_is_scaled_entropy():
    rng = np.random.default_rng(5)
    for n in (64, 512, 4096):
        e = np.round(rng.laplace(0, 300, n)).astype(np.int64)
        codes = np.clip(e + R, 1, 65535).astype(np.uint16)
        codes[rng.random(n) < 0.05] = 0
        c = np.bincount(codes, minlength=65536)
        c = c[c > 0].astype(np.float64)
        assert c.size > n // 4  # many symbols, most far beyond +-127
        H = -(c / n * np.log2(c / n)).sum()
        nqn = n * O.qlog(n)
        J = O.judge_j(codes)
        # each q() is rounded to an integer: |error| <= 0.5 per term, times c
        assert abs((nqn - J) / 2.0 ** 32 - n * H) <= (n + n) * 0.5 / 2.0 ** 32 + 1e-9 * n


@pytest.mark.parametrize("indep", [False, True])
def test_oracle_judge_flags_follow_block_scores(indep):
    x = synth.lognormal_grf((20, 27, 35), seed=31, decades=6, neg_frac=0.1, zero_frac=0.01)
    rng = np.random.default_rng(3)
    m = O.mlp_init(3, 16, seed=3)
    m["w1"] = (m["w1"] + rng.normal(0, 0.15, m["w1"].shape)).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.15, 16)).astype(np.float32)
    B = 8
    learned = O.compress(x, 1e-2, B, m, O.MODE_LEARNED, independent=indep)
    net = O.compress(x, 1e-2, B, m, O.MODE_PLAIN, independent=indep)
    lor = O.compress(x, 1e-2, B, None, O.MODE_LORENZO, independent=indep)
    nb = [-(-s // B) for s in x.shape]
    pos = 0
    seen = set()
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                size = 1
                for d, b in enumerate((bz, by, bx)):
                    size *= min(B, x.shape[d] - b * B)
                b = (bz * nb[1] + by) * nb[2] + bx
                sl = slice(pos, pos + size)
                flag = O.judge_j(net["codes"][sl]) > O.judge_j(lor["codes"][sl])
                assert learned["flags"][b] == int(flag)
                src = net if flag else lor
                assert np.array_equal(learned["codes"][sl], src["codes"][sl])
                assert learned["counts"][b] == np.count_nonzero(src["codes"][sl] == 0)
                seen.add(flag)
                pos += size
    assert pos == x.size
    assert seen == {False, True}  # both outcomes occur on this field
    xh, _ = O.decompress(learned["codes"], learned["raw"], learned["consts"], x.shape, x.dtype,
                         B, m, O.MODE_LEARNED, flags=learned["flags"], independent=indep)
    xd, hd = x.astype(np.float64), xh.astype(np.float64)
    nz = xd != 0
    assert np.all(hd[~nz] == 0)
    assert np.all(np.abs(xd[nz] - hd[nz]) <= 1e-2 * np.abs(xd[nz]))


def _one_unit(w, b1, v, b2, alpha):
    m = {"alpha": alpha, "w1": np.array([[w, 0.0], [0.0, 0.0]], dtype=np.float32),
         "b1": np.array([b1, 0.0], dtype=np.float32), "v": np.array([v, 0.0], dtype=np.float32),
         "b2": b2, "precision": 1}
    return m


def test_bf16_reference_hand_values():
    u = np.array([[1.0, 0.0]], dtype=np.float32)
    # w1 = 1 + 2^-8 is a tie between bf16 neighbours 1 and 1 + 2^-7: rounds to even (1)
    y, s = O.mlp_eval_bf16_ref(_one_unit(1.00390625, 0.0, 1.0, 0.0, 0.0), u)
    assert y[0] == 1.0 and s[0] < 1e-5
    # the hidden activation is rounded to bf16: 255.6 -> 256 (spacing 1 in [128, 256))
    y, _ = O.mlp_eval_bf16_ref(_one_unit(1.0, 0.6, 1.0, 0.0, 0.0),
                               np.array([[255.0, 0.0]], dtype=np.float32))
    assert y[0] == 256.0
    # alpha = 0.1: bf16(0.9f) = 0.8984375, bf16(0.1f) = 0.10009765625
    y, _ = O.mlp_eval_bf16_ref(_one_unit(1.0, 0.0, 1.0, 0.0, 0.1),
                               np.array([[10.0, 0.0], [-10.0, 0.0]], dtype=np.float32))
    assert y[0] == 0.8984375 * 10 + 0.10009765625 * 10
    assert y[1] == 0.10009765625 * -10
    # inputs are rounded to bf16 too: 257 -> 256 (tie to even), 259 -> 260
    y, _ = O.mlp_eval_bf16_ref(_one_unit(1.0, 0.0, 1.0, 0.5, 0.0),
                               np.array([[257.0, 0.0], [259.0, 0.0]], dtype=np.float32))
    assert y[0] == 256.5 and y[1] == 260.5


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_bf16_reference_reproduces_lorenzo(ndim, alpha):
    # with alpha in {0, 1} every weight of the Lorenzo-equivalent network is a
    # bf16 number and |z| < 256 keeps every activation exact
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, 8, alpha=alpha, seed=1)
    m["w1"][2:] = 0.0
    m["precision"] = 1
    rng = np.random.default_rng(ndim)
    u = rng.integers(-40, 41, size=(500, K)).astype(np.float32)
    coef = np.array([1 if bin(k + 2).count("1") % 2 else -1 for k in range(K)], dtype=np.float64)
    y, s = O.mlp_eval_bf16_ref(m, u)
    assert np.array_equal(y, u.astype(np.float64) @ coef)
    assert np.all(s < 1e-3)  # exact sums: only the FP32 allowance of layer 2 remains


def test_bf16_reference_slack_covers_a_rounding_flip():
    # far from a bf16 rounding boundary the slack is only the FP32 allowance
    m = _one_unit(1.0, 0.0, 1.0, 0.0, 0.0)
    y, s = O.mlp_eval_bf16_ref(m, np.array([[2.5, 0.0]], dtype=np.float32))
    assert y[0] == 2.5 and s[0] < 1e-5
    # z = 1 + 2^-8 + 2^-30: its FP32 value is the tie 1 + 2^-8, which rounds to
    # even (1.0); an FP32 sum a little above the tie would give 1 + 2^-7, so
    # the slack must cover that step
    m = _one_unit(1.0, 2.0 ** -8 + 2.0 ** -30, 1.0, 0.0, 0.0)
    y, s = O.mlp_eval_bf16_ref(m, np.array([[1.0, 0.0]], dtype=np.float32))
    assert y[0] == 1.0 and 2.0 ** -7 <= s[0] < 2.0 ** -6


# --- BF16 error bound ------------------------------------------------------------------------

def _bf16(a):
    """Round float32 values to bfloat16 (nearest even), numpy."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    r = ((b.astype(np.uint64) + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def _bf16_eval_unsplit(m, u):
    """A second admissible BF16 evaluation: bf16 weights and inputs, FP32 sums
    in reverse order, bf16(z), leaky ReLU on bf16(z), bf16(v) times it, FP32
    accumulation from the last unit down."""
    w1 = _bf16(np.asarray(m["w1"], np.float32))
    v = _bf16(np.asarray(m["v"], np.float32))
    a = np.float32(m["alpha"])
    out = np.zeros(u.shape[0])
    for i in range(u.shape[0]):
        ub = _bf16(u[i])
        y = np.float32(m["b2"])
        for j in reversed(range(len(m["b1"]))):
            z = np.float32(0.0)
            for k in reversed(range(u.shape[1])):
                z = np.float32(z + np.float32(w1[j, k] * ub[k]))
            z = np.float32(z + np.float32(m["b1"][j]))
            zb = _bf16(np.array([z]))[0]
            h = zb if zb >= 0 else np.float32(a * zb)
            y = np.float32(y + np.float32(v[j] * _bf16(np.array([h]))[0]))
        out[i] = float(y)
    return out


@pytest.mark.parametrize("ndim,H", [(3, 32), (3, 16), (2, 16)])
def test_bf16_bound_covers_admissible_evaluations(ndim, H):
    rng = np.random.default_rng(ndim * 100 + H)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=ndim)
    m["w1"] = (m["w1"] + rng.normal(0, 0.3, (H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 2.0, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.3, H)).astype(np.float32)
    m["b2"] = float(np.float32(0.7))
    u = np.concatenate([rng.integers(-40, 41, (300, K)),
                        rng.integers(-3000, 3001, (300, K))]).astype(np.float32)
    y, bound = O.mlp_eval_f64(m, u)
    mag = np.abs(u.astype(np.float64)) @ np.abs(m["w1"]).T.astype(np.float64)
    scale = (mag + np.abs(m["b1"])) @ np.abs(m["v"]).astype(np.float64) + abs(m["b2"])
    # the FP32 network is the same function up to FP32 roundings
    y32 = O.mlp_eval(m, u).astype(np.float64)
    assert np.all(np.abs(y32 - y) <= 2.0 ** -18 * scale)
    yr, _ = O.mlp_eval_bf16_ref(dict(m, precision=1), u)
    assert np.all(np.abs(yr - y) <= bound)
    yu = _bf16_eval_unsplit(m, u[::7])
    assert np.all(np.abs(yu - y[::7]) <= bound[::7])
    # the bound is a few bf16 units of the network's magnitudes, not more
    assert np.all(bound <= 2.0 ** -5 * scale + 1e-12)


def test_bf16_bound_is_tight_where_roundings_line_up():
    # w = (1 + 2^-8, -1), u = (257, 256): 1 + 2^-8 rounds to 1 and 257 to 256
    # (ties to even), so the first product loses 2.004 while the second is
    # exact and cancels the rest: z = 2.004 exactly, the BF16 evaluation gives
    # 0.  The bound's first-layer term (2U + U^2) S, S = 514, is what covers
    # it; the terms proportional to |z| are 100 times smaller.
    m = {"alpha": 0.0, "w1": np.array([[1.00390625, -1.0], [0.0, 0.0]], dtype=np.float32),
         "b1": np.zeros(2, dtype=np.float32), "v": np.array([1.0, 0.0], dtype=np.float32),
         "b2": 0.0, "precision": 1}
    u = np.array([[257.0, 256.0]], dtype=np.float32)
    y, bound = O.mlp_eval_f64(m, u)
    yr, _ = O.mlp_eval_bf16_ref(m, u)
    assert y[0] == 1.00390625 * 257 - 256 and yr[0] == 0.0
    err = abs(yr[0] - y[0])
    assert err <= bound[0] <= 2.5 * err
    # the rounding of z: 255.6 becomes 256 (spacing 1 in [128, 256)); every
    # weight and input exact, so only the z rounding and the scalings remain
    m = _one_unit(1.0, 0.6, 1.0, 0.0, 0.0)
    u = np.array([[255.0, 0.0]], dtype=np.float32)
    y, bound = O.mlp_eval_f64(m, u)
    yr, _ = O.mlp_eval_bf16_ref(m, u)
    err = abs(yr[0] - y[0])
    assert err == pytest.approx(0.4, abs=1e-6)
    assert err <= bound[0] <= 12 * err  # it assumes w and u might round too
    # every operand a bf16 number and |z| < 256: bound of rounding-free sums only
    m = _one_unit(0.5, 0.25, -1.5, 0.0, 0.0)
    y, bound = O.mlp_eval_f64(m, np.array([[12.0, 0.0]], dtype=np.float32))
    assert y[0] == -1.5 * 6.25
    assert bound[0] <= 2 ** -6 * 12.0
