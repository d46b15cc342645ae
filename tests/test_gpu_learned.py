"""GPU checks of the learned path (Sec. 4.2 / 4.3) against the CPU oracle.

- sampling: the drawn pairs (point index, inputs, target, split flag) are
  bit-identical to the oracle's, in 1-D/2-D/3-D, FP32/FP64, halo and
  independent blocks;
- loss and gradient of the FP32 device trainer against the oracle's FP64
  ones, and three Adam steps against the oracle's Adam;
- the end-to-end training entry point: pair counts, scale, the validation
  score of the untrained and of the returned network equal to the oracle's
  scores of those networks, the choice is the best score, and it pays;
- the matrix-core (BF16) network inside the codec: points without a full
  stencil carry exactly the oracle's Lorenzo codes; at every other point the
  integer prediction the code implies lies within 1/2 + B(u) of the network's
  FP64 value (the FP32-weight network of Sec. 4.2 evaluated exactly), B(u) the
  oracle's error bound for BF16-operand inference derived from bf16 unit
  roundoff and the weight and input magnitudes; as a secondary check, within
  1/2 + slack of the oracle's reference of the kernel's own rounding points;
  the stream decodes bit-exactly to the value its codes define (the inverse
  transform of the grid value, or the stored raw value);
- the per-block judge: with FP32 networks every output equals the oracle's
  learned mode (entropy of each block's full code multiset); with the BF16
  network every block's flag is the comparison of the two scores of that
  block (network codes of the plain run, Lorenzo codes of the oracle) and the
  block carries the winner's codes;
- 512^3 FP32: train, compress with the judge, decode; bound on every point,
  sampled codes against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth
from tests.test_gpu_codec import _case as codec_case

pytestmark = pytest.mark.gpu

R = 32768


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_model(ndim, H, seed, scale=0.2, precision=1):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, scale, size=(H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 0.5, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, scale, H)).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal(0, 0.3)))
    m["precision"] = precision
    return m


def stream_order(shape, B):
    """Field index of every stream position, and the size of every block."""
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    nb = [-(-s // B) for s in shape]
    parts = [idx[tuple(slice(b * B, (b + 1) * B) for b in bc)].ravel() for bc in np.ndindex(*nb)]
    return np.concatenate(parts), np.array([len(p) for p in parts])


def net_points(shape, B, indep):
    """Points whose every neighbour exists (the network applies there)."""
    m = np.ones(shape, dtype=bool)
    for d, c in enumerate(np.indices(shape)):
        m &= ((c % B) if indep else c) > 0
    return m


def stencil_inputs(p):
    """u_k = n_{k+2} - n_1 at every point with a full stencil (others: junk),
    neighbour o = one step back along the axes of its bits (bit 0 = fastest)."""
    D = p.ndim
    K = (1 << D) - 2
    pp = np.pad(p.astype(np.int64), [(1, 0)] * D)

    def nb(o):
        sl = []
        for d in range(D):
            back = (o >> (D - 1 - d)) & 1
            sl.append(slice(1 - back, pp.shape[d] - back))
        return pp[tuple(sl)]

    n1 = nb(1)
    u = np.stack([nb(k + 2) - n1 for k in range(K)], -1) if K else np.zeros(p.shape + (0,))
    return u, n1


def check_bf16_stream(x, eps, B, model, indep, stream):
    """Checks of a plain (no judge) matrix-core stream; returns its codes in
    field order."""
    sec = pwrel.sections(stream)
    codes_s = sec["codes"].cpu().numpy().view(np.uint16)
    counts = sec["counts"].cpu().numpy().view(np.uint32)
    raw = sec["raw"].cpu().numpy()
    order, sizes = stream_order(x.shape, B)
    codes = np.empty_like(codes_s)
    codes[order] = codes_s
    codes = codes.reshape(x.shape)
    ref = O.compress(x, eps, B, model, O.MODE_PLAIN, independent=indep)
    rc = np.empty_like(ref["codes"])
    rc[order] = ref["codes"]
    rc = rc.reshape(x.shape)
    p = ref["p"]
    net = net_points(x.shape, B, indep)
    # no full stencil: Lorenzo with missing neighbours as zero, exactly
    assert np.array_equal(codes[~net], rc[~net])
    # full stencil: the implied integer prediction against the network's FP64
    # value, within the derived BF16 bound (primary), and against the
    # reference of the kernel's rounding points (secondary)
    u, n1 = stencil_inputs(p)
    un = u[net].astype(np.float32)
    y64, bound = O.mlp_eval_f64(model, un)
    yref, slack = O.mlp_eval_bf16_ref(model, un)
    c = codes[net].astype(np.int64)
    pn, n1n = p[net].astype(np.int64), n1[net]
    coded = c != 0
    y_int = c - R + pn - n1n
    dev64 = np.abs(y_int[coded] - y64[coded])
    assert np.all(dev64 <= 0.5 + bound[coded]), (dev64 - bound[coded]).max()
    dev_ = np.abs(y_int[coded] - yref[coded])
    assert np.all(dev_ <= 0.5 + slack[coded] + 1e-9), dev_.max()
    # balance points at full stencils: failed verification or an error near 2^15
    for i in np.flatnonzero(~coded):
        xi = x[net].reshape(-1)[i]
        xh = O.inverse_field(np.array([pn[i]], dtype=np.int32), ref["consts"], x.dtype)[0]
        near = abs(yref[i] + n1n[i] - pn[i]) >= R - 1 - slack[i]
        assert near or not O.verify(xi, xh, eps)
    # counts and raw values follow the codes
    bstart = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    assert np.array_equal(counts, np.add.reduceat((codes_s == 0).astype(np.int64), bstart))
    zf = order[codes_s == 0]
    assert np.array_equal(raw.view(np.uint8), x.reshape(-1)[zf].view(np.uint8))
    return codes


def expected_xh(x, codes, p, consts):
    inv = O.inverse_field(p, consts, x.dtype)
    return np.where(codes == 0, x, inv)


# --- sampling -----------------------------------------------------------------------------

SAMPLE_CASES = {
    "grf3d_halo": (lambda: synth.lognormal_grf((40, 44, 52), seed=21), 1e-2, 8, False, 0.1),
    "grf3d_indep": (lambda: synth.lognormal_grf((40, 44, 52), seed=21), 1e-2, 8, True, 0.1),
    "bumps3d_f64": (lambda: synth.gaussian_bumps((30, 33, 35), seed=22, zero_frac=0.02,
                                                 dtype=np.float64), 1e-3, 8, False, 0.3),
    "zonal2d": (lambda: synth.zonal_bands_2d((90, 130), seed=23), 1e-2, 16, False, 0.2),
    "grf2d_indep": (lambda: synth.lognormal_grf((90, 130), seed=24), 1e-2, 16, True, 0.2),
    "grf1d": (lambda: synth.lognormal_grf((50000,), seed=25), 1e-2, 256, False, 0.1),
}


@pytest.mark.parametrize("name", list(SAMPLE_CASES))
def test_sample_matches_oracle(ctx, name):
    make, eps, B, indep, rho = SAMPLE_CASES[name]
    x = make()
    seed = 1234 + len(name)
    idx, u, t, iv = ctx.sample(dev(x), eps, B, independent=indep, rho=rho, seed=seed)
    c = O.consts(x, eps)
    ref = O.sample(O.transform_field(x, c), c, B, rho, seed, independent=indep)
    assert idx.numel() == ref["idx"].size > 0
    assert np.array_equal(idx.cpu().numpy().astype(np.uint64), ref["idx"])
    assert np.array_equal(u.cpu().numpy(), ref["u"])
    assert np.array_equal(t.cpu().numpy(), ref["t"])
    assert np.array_equal(iv.cpu().numpy().astype(bool), ref["is_val"])


# --- loss, gradient, Adam ---------------------------------------------------------------------

def _pairs(ndim, n, seed):
    shape = {3: (40, 40, 40), 2: (200, 200), 1: (40000,)}[ndim]
    x = synth.lognormal_grf(shape, seed=seed)
    c = O.consts(x, 1e-2)
    s = O.sample(O.transform_field(x, c), c, 8 if ndim == 3 else (16 if ndim == 2 else 256),
                 0.5, seed)
    assert s["t"].size >= n
    return s["u"][:n].astype(np.float32), s["t"][:n].astype(np.float32)


@pytest.mark.parametrize("ndim,H", [(3, 16), (3, 32), (2, 8), (1, 4)])
def test_loss_grad_matches_oracle(ctx, ndim, H):
    K = (1 << ndim) - 2
    u, t = _pairs(ndim, 3000, 40 + ndim)
    rng = np.random.default_rng(H)
    th = rng.normal(0, 0.3, H * K + 2 * H + 1).astype(np.float32)
    sigma, lam, alpha = 7.3, 1e-3, 0.01
    loss, g = ctx.loss_grad(dev(th), H, K, alpha, dev(u), dev(t), sigma, lam)
    th64, u64, t64 = th.astype(np.float64), u.astype(np.float64), t.astype(np.float64)
    loss_r, g_r = O.loss_grad(th64, H, K, alpha, u64, t64, sigma, lam)
    gabs, gres = O.loss_grad_abs(th64, H, K, alpha, u64, t64, sigma, lam)
    assert abs(loss - loss_r) <= 1e-5 * abs(loss_r)
    g = g.cpu().numpy().astype(np.float64)
    # FP32 attainable: each component is a serial FP32 sum of n terms (error
    # <= gamma_n sum |terms|, the recursive-summation bound), each term a few
    # roundings off, and the residual it multiplies off by a small multiple of
    # the magnitudes it was computed from
    n, u32 = t.size, 2.0 ** -24
    tol = u32 * ((n + 16) * gabs + (H + K + 16) * gres)
    d = np.abs(g - g_r)
    assert np.all(d <= tol), (d / tol).max()
    # and typically far inside it (rounding errors do not all line up)
    assert np.median(d / tol) <= 0.05, np.median(d / tol)


@pytest.mark.parametrize("ndim,H", [(3, 16), (2, 8)])
def test_adam_steps_match_oracle(ctx, ndim, H):
    K = (1 << ndim) - 2
    u, t = _pairs(ndim, 3 * 256, 50 + ndim)
    m = random_model(ndim, H, 5, precision=0)
    th0 = O.theta_from_model(m).astype(np.float32)
    sigma, alpha = float(np.sqrt(np.mean(t.astype(np.float64) ** 2))), m["alpha"]
    lrs, lams = [1e-3, 3e-3], [1e-4, 0.0]
    out = ctx.train_pairs(dev(u), dev(t), H, K, alpha, sigma, dev(th0), lrs, lams, batch=256,
                          epochs=1).cpu().numpy().astype(np.float64)
    u64, t64 = u.astype(np.float64), t.astype(np.float64)
    for c in range(2):
        ref, *_ = O.train_pass(th0.astype(np.float64), H, K, alpha, u64, t64, sigma, lams[c],
                               lrs[c], 256, 1)
        d = np.abs(out[c] - ref)
        # Adam's step lr m^ / (sqrt(v^) + eps) depends on gradient ratios, not
        # sizes: a parameter whose gradient stays well above its FP32 error at
        # every step follows the oracle to a small fraction of lr; one whose
        # gradient is at the rounding level may take another sign.  Replay the
        # oracle step by step and split the parameters that way.
        th, am, av, st = th0.astype(np.float64), None, None, 0
        clear = np.ones(th.size, dtype=bool)
        for s0 in range(0, t.size, 256):
            ub, tb = u64[s0:s0 + 256], t64[s0:s0 + 256]
            _, gs = O.loss_grad(th, H, K, alpha, ub, tb, sigma, lams[c])
            ga, gr = O.loss_grad_abs(th, H, K, alpha, ub, tb, sigma, lams[c])
            tol = 2.0 ** -24 * ((tb.size + 16) * ga + (H + K + 16) * gr)
            clear &= np.abs(gs) > 20 * tol
            th, am, av, st = O.train_pass(th, H, K, alpha, ub, tb, sigma, lams[c], lrs[c], 256,
                                          1, am, av, st)
        assert np.array_equal(th, ref)
        assert clear.mean() >= 0.9, clear.mean()
        assert np.all(d[clear] <= 1e-3 * lrs[c]), d[clear].max() / lrs[c]
        assert np.median(d) <= 1e-4 * lrs[c]


# --- training entry point ----------------------------------------------------------------------

@pytest.fixture(scope="module")
def grf64():
    return synth.lognormal_grf((64, 64, 64), seed=1001, decades=8, neg_frac=0.1, zero_frac=0.005)


def test_train_entry_point(ctx, grf64):
    x = grf64
    init = O.mlp_init(3, 16, seed=7)
    model, rep = ctx.train(dev(x), 1e-2, 8, init=init, rho=0.1, seed=99, precision=1)
    c = O.consts(x, 1e-2)
    s = O.sample(O.transform_field(x, c), c, 8, 0.1, 99)
    uv, tv = s["u"][s["is_val"]], s["t"][s["is_val"]]
    tt = s["t"][~s["is_val"]].astype(np.float64)
    assert rep["n_val"] == tv.size and rep["n_train"] == tt.size
    assert abs(rep["sigma"] - max(1.0, np.sqrt(np.mean(tt ** 2)))) <= 1e-12 * rep["sigma"]
    assert rep["n_candidates"] == 10
    sc = rep["val_score"]
    assert sc[0] == O.val_score(init, uv, tv)
    assert rep["chosen"] == int(np.argmax(sc))
    assert sc[rep["chosen"]] == O.val_score(model, uv, tv)
    assert model["precision"] == 1
    gain = (sc[rep["chosen"]] - sc[0]) / 2.0 ** 32 / tv.size
    assert rep["chosen"] > 0 and gain > 0.2, gain
    # the trained network compresses the field better than Lorenzo
    xd = dev(x)
    bits = []
    for net in (False, True):
        st = ctx.compress(xd, 1e-2, 8, model, use_net=net)
        bits.append(pwrel.huffman_bits(ctx.histogram(pwrel.sections(st)["codes"]))[0])
    assert bits[1] < bits[0], bits


# --- matrix-core network in the codec -------------------------------------------------------

BF16_CASES = {
    "grf_ragged": (lambda: synth.lognormal_grf((37, 45, 51), seed=2), 1e-3, 8, False, (3, 16, 1)),
    "grf_ragged_indep": (lambda: synth.lognormal_grf((37, 45, 51), seed=2), 1e-3, 8, True,
                         (3, 16, 1)),
    "grf_B4_H32": (lambda: synth.lognormal_grf((24, 28, 90), seed=3), 1e-2, 4, False, (3, 32, 2)),
    "grf_B16_H8": (lambda: synth.lognormal_grf((40, 50, 70), seed=4), 1e-2, 16, False, (3, 8, 4)),
    "grf_B5": (lambda: synth.lognormal_grf((21, 22, 23), seed=5), 1e-2, 5, False, (3, 16, 5)),
    "zonal_2d": (lambda: synth.zonal_bands_2d((150, 301), seed=6), 1e-2, 16, False, (2, 16, 6)),
    "f64_1e-4": (lambda: synth.lognormal_grf((24, 40, 50), seed=9, decades=12, neg_frac=0.1,
                                              zero_frac=0.01, dtype=np.float64), 1e-4, 8, False,
                 (3, 16, 9)),
    # independent blocks decoded one per lane (matrix cores for 64 blocks at once)
    "lanes_B8_indep": (lambda: synth.lognormal_grf((72, 64, 136), seed=23), 1e-2, 8, True,
                       (3, 32, 23)),
    "lanes_B4_indep": (lambda: synth.lognormal_grf((30, 41, 53), seed=24), 1e-2, 4, True,
                       (3, 32, 24)),
    "lanes_2d_indep": (lambda: synth.zonal_bands_2d((150, 301), seed=25), 1e-2, 16, True,
                       (2, 32, 25)),
    "lanes_f64_indep": (lambda: synth.lognormal_grf((24, 40, 50), seed=26, decades=12,
                                                     neg_frac=0.1, zero_frac=0.01,
                                                     dtype=np.float64), 1e-4, 8, True,
                        (3, 16, 26)),
}


@pytest.mark.parametrize("name", list(BF16_CASES))
def test_bf16_codec(ctx, name):
    make, eps, B, indep, (nd, H, ms) = BF16_CASES[name]
    x = make()
    model = random_model(nd, H, ms)
    stream = ctx.compress(dev(x), eps, B, model, independent=indep)
    codes = check_bf16_stream(x, eps, B, model, indep, stream)
    c = O.consts(x, eps)
    p = O.transform_field(x, c)
    xh = ctx.decompress(stream).cpu().numpy()
    assert np.array_equal(xh.view(np.uint8), expected_xh(x, codes, p, c).view(np.uint8))


def _judge_case(name):
    if name == "grf_random":
        return synth.lognormal_grf((37, 45, 51), seed=12, decades=6, neg_frac=0.1,
                                   zero_frac=0.01), 1e-2, 8, random_model(3, 16, 12, 0.15), False
    if name == "grf_random_indep":
        return synth.lognormal_grf((37, 45, 51), seed=12, decades=6, neg_frac=0.1,
                                   zero_frac=0.01), 1e-2, 8, random_model(3, 16, 12, 0.15), True
    if name == "grf_thin":  # one pencil row in z, ragged in every axis
        return synth.lognormal_grf((5, 19, 61), seed=12, decades=6, neg_frac=0.1,
                                   zero_frac=0.01), 1e-2, 8, random_model(3, 16, 12, 0.15), False
    if name == "grf_B4":
        return synth.lognormal_grf((20, 24, 44), seed=13), 1e-2, 4, random_model(3, 32, 13, 0.1), \
            False
    if name == "zonal_2d":
        return synth.zonal_bands_2d((150, 301), seed=14), 1e-2, 16, random_model(2, 16, 14, 0.1), \
            False
    if name.startswith("wide_span"):  # grid values spanning more than 2^27: 64-bit branch
        x, eps, B, _, indep = codec_case(name)
        return x, eps, B, random_model(3, 16, 12, 0.15), indep
    raise KeyError(name)


JUDGE_CASES = ["grf_random", "grf_random_indep", "grf_thin", "grf_B4", "zonal_2d",
               "wide_span_halo", "wide_span_indep"]


@pytest.mark.parametrize("name", JUDGE_CASES)
def test_judge_fp32_bit_exact(ctx, name):
    x, eps, B, model, indep = _judge_case(name)
    model = dict(model, precision=0)
    stream = ctx.compress(dev(x), eps, B, model, judge=True, independent=indep)
    sec = pwrel.sections(stream)
    ref = O.compress(x, eps, B, model, O.MODE_LEARNED, independent=indep)
    assert np.array_equal(sec["codes"].cpu().numpy().view(np.uint16), ref["codes"])
    assert np.array_equal(sec["counts"].cpu().numpy().view(np.uint32), ref["counts"])
    assert np.array_equal(sec["bflags"].cpu().numpy(), ref["flags"])
    assert np.array_equal(sec["raw"].cpu().numpy().view(np.uint8), ref["raw"].view(np.uint8))
    assert 0 < ref["flags"].sum() < ref["flags"].size
    xh = ctx.decompress(stream).cpu().numpy()
    rxh, _ = O.decompress(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, B, model,
                          O.MODE_LEARNED, flags=ref["flags"], independent=indep)
    assert np.array_equal(xh.view(np.uint8), rxh.view(np.uint8))


@pytest.mark.parametrize("name", JUDGE_CASES)
def test_judge_bf16(ctx, name):
    x, eps, B, model, indep = _judge_case(name)
    xd = dev(x)
    plain = ctx.compress(xd, eps, B, model, independent=indep).clone()
    check_bf16_stream(x, eps, B, model, indep, plain)
    judged = ctx.compress(xd, eps, B, model, judge=True, independent=indep)
    net_codes = pwrel.sections(plain)["codes"].cpu().numpy().view(np.uint16)
    sec = pwrel.sections(judged)
    codes = sec["codes"].cpu().numpy().view(np.uint16)
    flags = sec["bflags"].cpu().numpy()
    counts = sec["counts"].cpu().numpy().view(np.uint32)
    lor = O.compress(x, eps, B, None, O.MODE_LORENZO, independent=indep)["codes"]
    order, sizes = stream_order(x.shape, B)
    pos = 0
    for b, n in enumerate(sizes):
        sl = slice(pos, pos + n)
        flag = O.judge_j(net_codes[sl]) > O.judge_j(lor[sl])
        assert flags[b] == int(flag), b
        assert np.array_equal(codes[sl], net_codes[sl] if flag else lor[sl]), b
        assert counts[b] == np.count_nonzero(codes[sl] == 0)
        pos += n
    assert 0 < flags.sum() < flags.size
    raw = sec["raw"].cpu().numpy()
    assert np.array_equal(raw.view(np.uint8), x.reshape(-1)[order[codes == 0]].view(np.uint8))
    fcodes = np.empty_like(codes)
    fcodes[order] = codes
    c = O.consts(x, eps)
    xh = ctx.decompress(judged).cpu().numpy()
    exp = expected_xh(x, fcodes.reshape(x.shape), O.transform_field(x, c), c)
    assert np.array_equal(xh.view(np.uint8), exp.view(np.uint8))


# --- full size: 512^3 FP32, trained BF16 network with the judge -------------------------------

def test_learned_full_size_512cubed(ctx):
    x = synth.lognormal_grf((512, 512, 512), seed=1001)
    xd = dev(x)
    eps, B = 1e-2, 8
    model, rep = ctx.train(xd, eps, B, rho=0.01, seed=1001, hidden=32, precision=1)
    assert rep["chosen"] > 0
    stream = ctx.compress(xd, eps, B, model, judge=True)
    sec = pwrel.sections(stream)
    h = sec["header"]
    codes = sec["codes"].cpu().numpy().view(np.uint16)
    counts = sec["counts"].cpu().numpy().view(np.uint32)
    flags = sec["bflags"].cpu().numpy()
    raw = sec["raw"].cpu().numpy()
    assert flags.mean() > 0.5
    c = O.consts(x, eps)
    # sampled points: codes of Lorenzo blocks exactly; network blocks within the BF16 slack
    rng = np.random.default_rng(7)
    idx = rng.choice(x.size, 100000, replace=False)
    zz, yy, xx = np.unravel_index(idx, x.shape)
    b = ((zz // B) * 64 + yy // B) * 64 + xx // B
    lor = O.codes_at(x, c, B, idx, None, O.MODE_LORENZO)
    pos = lor["pos"].astype(np.int64)
    fl = flags[b] == 1
    assert np.array_equal(codes[pos[~fl]], lor["codes"][~fl])
    full = fl & (zz > 0) & (yy > 0) & (xx > 0)
    sel = idx[full]
    net = O.codes_at(x, c, B, sel, model, O.MODE_PLAIN)
    left = O.codes_at(x, c, B, sel - 1, None, O.MODE_LORENZO)
    cg = codes[net["pos"].astype(np.int64)].astype(np.int64)
    coded = cg != 0
    y_int = cg - R + net["p"].astype(np.int64) - left["p"].astype(np.int64)
    d64 = np.abs(y_int[coded] - net["y64"][coded])
    assert np.all(d64 <= 0.5 + net["bound"][coded]), (d64 - net["bound"][coded]).max()
    d = np.abs(y_int[coded] - net["yref"][coded])
    assert np.all(d <= 0.5 + net["slack"][coded] + 1e-9), d.max()
    # network blocks at faces (no full stencil) use Lorenzo with missing neighbours as zero
    face = fl & ~full
    assert np.array_equal(codes[pos[face]], lor["codes"][face])
    # balance points: counts and raw values in stream order
    zpos = np.flatnonzero(codes == 0)
    assert counts.sum() == zpos.size == h["n_raw"]
    order_first = zpos[:20000]
    # field index of stream positions (blocks of 8^3, all full at 512^3)
    blk, loc = order_first // 512, order_first % 512
    bz, by, bx = blk // 4096, (blk // 64) % 64, blk % 64
    lz, ly, lx = loc // 64, (loc // 8) % 8, loc % 8
    fi = ((bz * 8 + lz) * 512 + by * 8 + ly) * 512 + bx * 8 + lx
    assert np.array_equal(raw[:fi.size].view(np.uint32), x.reshape(-1)[fi].view(np.uint32))
    # reconstruction: bound on every point
    xh = ctx.decompress(stream)
    hd, xt = xh.double(), xd.double()
    z = xt == 0
    assert bool(torch.all(hd[z] == 0))
    assert bool(torch.all(torch.signbit(hd[~z]) == torch.signbit(xt[~z])))
    assert bool(torch.all((xt - hd).abs() <= eps * xt.abs()))
