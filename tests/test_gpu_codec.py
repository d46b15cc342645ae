"""GPU parity of the HIP codec against the CPU oracle (run on an MI355X).

Bar: bit-exact for every integer/byte output (grid values, codes, per-block
counts, raw-value lists, header constants) and for the reconstruction
(x^ is a function of the grid value only), on fields that span several tiles
with ragged edges, in 1-D/2-D/3-D, FP32/FP64, halo and independent blocks,
and at the full 512^3 size on sampled points plus whole-field invariants.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth

pytestmark = pytest.mark.gpu

CONST_KEYS = ("eps0", "b_a", "w", "r", "Lp", "Ln", "d0", "p_zero", "b_sign", "n_lo", "delta")


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host_sections(stream):
    sec = pwrel.sections(stream)
    return {"h": sec["header"],
            "codes": sec["codes"].cpu().numpy().view(np.uint16),
            "counts": sec["counts"].cpu().numpy().view(np.uint32),
            "raw": sec["raw"].cpu().numpy(),
            "model": sec.get("model")}


def random_model(ndim, H, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, scale, size=(H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 0.5, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, scale, H)).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal(0, 0.3)))
    return m


def assert_bound(x, xh, eps):
    xd, hd = x.astype(np.float64), xh.astype(np.float64)
    z = xd == 0
    assert np.all(hd[z] == 0)
    assert np.all(np.signbit(hd[~z]) == np.signbit(xd[~z]))
    assert np.all(np.abs(xd[~z] - hd[~z]) <= eps * np.abs(xd[~z]))


# --- deterministic math ----------------------------------------------------------

def test_detmath_bit_identical_to_oracle(ctx):
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        np.ldexp(1.0 + rng.random(20000), rng.integers(-1074, 1023, 20000)),
        np.ldexp(1.0, np.arange(-1074, 1024)).astype(np.float64),
        rng.random(2000) * 2.0 ** -1022,                      # subnormals
        1.0 + (rng.random(2000) - 0.5) * 1e-12,
        np.array([1.4142135623730951, np.nextafter(1.4142135623730951, 2), 5e-324]),
    ])
    xs = xs[np.isfinite(xs) & (xs > 0)]
    l2, _ = ctx.detmath(dev(xs))
    ts = np.concatenate([rng.uniform(-1100, 1030, 20000), rng.uniform(-1075, -1020, 5000),
                         np.arange(-1080, 1030).astype(np.float64) + 0.5,
                         rng.uniform(-3, 3, 5000)])
    _, e2 = ctx.detmath(dev(ts))
    ref_l = O.det_log2(xs)
    ref_e = O.det_exp2(ts)
    assert np.array_equal(l2.cpu().numpy().view(np.uint64), ref_l.view(np.uint64))
    assert np.array_equal(e2.cpu().numpy().view(np.uint64), ref_e.view(np.uint64))


# --- transform (a1-a3) -------------------------------------------------------------

@pytest.mark.parametrize("case", ["bumps_f32", "grf_f64_subnormal", "grf_f32_1e-3"])
def test_transform_and_constants_match_oracle(ctx, case):
    if case == "bumps_f32":
        x, eps = synth.gaussian_bumps((64, 64, 64), seed=1000, zero_frac=0.01), 1e-2
    elif case == "grf_f64_subnormal":
        x = synth.lognormal_grf((24, 40, 50), seed=5, decades=12, neg_frac=0.1,
                                zero_frac=0.01, dtype=np.float64)
        x.reshape(-1)[::997] = 3e-320
        eps = 1e-4
    else:
        x, eps = synth.lognormal_grf((33, 65, 130), seed=6), 1e-3
    p, h = ctx.transform(dev(x), eps)
    c = O.consts(x, eps)
    for k in CONST_KEYS:
        assert h[k] == c[k], k
    assert np.array_equal(p.cpu().numpy(), O.transform_field(x, c))


# --- prediction on a given grid field (a4-a5) ------------------------------------------

@pytest.mark.parametrize("shape,B", [((37, 29, 41), 8), ((16, 16, 16), 4), ((20, 33, 17), 16),
                                     ((70, 131), 16), ((5000,), 64), ((19, 23, 29), 5)])
@pytest.mark.parametrize("net", ["lorenzo", "random"])
@pytest.mark.parametrize("indep", [False, True])
def test_encode_grid_matches_oracle(ctx, shape, B, net, indep):
    rng = np.random.default_rng(abs(hash((shape, B))) % 1000)
    p = np.cumsum(rng.integers(-40, 41, size=shape), axis=-1).astype(np.int32)
    model = None if net == "lorenzo" else random_model(len(shape), 16, 3)
    got = ctx.encode_grid(dev(p), B, model, use_net=model is not None, independent=indep)
    ref = O.encode_p(p, B, model, use_net=model is not None, independent=indep)
    assert np.array_equal(got.cpu().numpy().view(np.uint16), ref)


def test_encode_grid_annihilation(ctx):
    rng = np.random.default_rng(11)
    nz, ny, nx = 33, 40, 70
    g = rng.integers(-5000, 5000, size=(ny, nx))
    h = rng.integers(-5000, 5000, size=(nz, nx))
    k = rng.integers(-5000, 5000, size=(nz, ny))
    p = (g[None] + h[:, None] + k[:, :, None]).astype(np.int32)
    codes = ctx.encode_grid(dev(p), 8, None, use_net=False).cpu().numpy().view(np.uint16)
    pos = O.codes_at(np.ones(p.shape, np.float32), O.consts(np.ones(4, np.float32), 0.01), 8,
                     np.arange(p.size), None, O.MODE_LORENZO)["pos"].astype(np.int64)
    zz, yy, xx = np.unravel_index(np.arange(p.size), p.shape)
    interior = (zz > 0) & (yy > 0) & (xx > 0)
    assert np.all(codes[pos[interior]] == 32768)


# --- full codec (a1-a8) -------------------------------------------------------------------

def _case(name):
    if name == "config0_bumps64":
        x = synth.gaussian_bumps((64, 64, 64), seed=1000, zero_frac=0.01)
        c = O.consts(x, 1e-2)
        model, *_ = O.train_rule(O.transform_field(x, c), c, 8, O.mlp_init(3, 16, seed=1000),
                                 rho=0.10, seed=1000)
        return x, 1e-2, 8, model, False
    if name == "grf_ragged_1e-3":
        return synth.lognormal_grf((37, 45, 51), seed=2), 1e-3, 8, random_model(3, 16, 1), False
    if name == "grf_ragged_indep":
        return synth.lognormal_grf((37, 45, 51), seed=2), 1e-3, 8, random_model(3, 16, 1), True
    if name == "grf_B4_H32":
        return synth.lognormal_grf((24, 28, 90), seed=3), 1e-2, 4, random_model(3, 32, 2), False
    if name == "grf_B16_H8":
        return synth.lognormal_grf((40, 50, 70), seed=4), 1e-2, 16, random_model(3, 8, 4), False
    if name == "grf_B5":
        return synth.lognormal_grf((21, 22, 23), seed=5), 1e-2, 5, random_model(3, 16, 5), False
    if name == "zonal_2d":
        x = synth.zonal_bands_2d((150, 301), seed=6)
        return x, 1e-2, 16, random_model(2, 16, 6), False
    if name == "grf_2d_B64":
        return synth.lognormal_grf((130, 200), seed=7), 1e-2, 64, random_model(2, 16, 7), False
    if name == "grf_1d_halo":
        return synth.lognormal_grf((10007,), seed=8), 1e-2, 256, random_model(1, 8, 8), False
    if name == "grf_1d_indep":
        return synth.lognormal_grf((10007,), seed=8), 1e-2, 256, random_model(1, 8, 8), True
    if name == "f64_1e-4":
        x = synth.lognormal_grf((24, 40, 50), seed=9, decades=12, neg_frac=0.1, zero_frac=0.01,
                                dtype=np.float64)
        x.reshape(-1)[::991] = 7e-321
        return x, 1e-4, 8, random_model(3, 16, 9), False
    if name.startswith("f32_range_ends"):
        # magnitudes across the whole FP32 range, with extra mass at the edges
        # of the fast paths' certified range (2^-124, 2^126), a few subnormals,
        # zeros and both signs
        rng = np.random.default_rng(11)
        n = 20 * 24 * 30
        e = rng.uniform(-126.0, 127.9, n)
        pick = rng.random(n)
        e[pick < 0.15] = rng.uniform(-126.0, -122.0, int((pick < 0.15).sum()))
        m = (pick >= 0.15) & (pick < 0.30)
        e[m] = rng.uniform(124.0, 127.9, int(m.sum()))
        m = (pick >= 0.30) & (pick < 0.32)
        e[m] = rng.uniform(-140.0, -126.5, int(m.sum()))
        x = (np.exp2(e) * np.where(rng.random(n) < 0.3, -1.0, 1.0)).astype(np.float32)
        x[rng.random(n) < 0.01] = 0.0
        return x.reshape(20, 24, 30), 1e-2, 8, random_model(3, 16, 11), False
    if name.startswith("f32_smooth_range"):
        # a smooth field over 75 decades (every point coded at 1e-2), shifted
        # across the upper or the lower edge of the certified range
        x = synth.lognormal_grf((20, 24, 30), seed=12, decades=75, neg_frac=0.3, zero_frac=0.01)
        x = (x * (8.0 if name.endswith("hi") else 2.0 ** -6)).astype(np.float32)
        return x, 1e-2, 8, random_model(3, 16, 12), False
    if name.startswith("wide_span"):
        # a smooth field plus a few magnitudes near both ends of the FP32
        # range: at a bound of 5e-7 the grid values span more than 2^27, so the
        # kernels take their 64-bit (generic) branch; about a fifth of the
        # points end raw
        rng = np.random.default_rng(14)
        x = synth.lognormal_grf((20, 24, 30), seed=14, decades=0.05, neg_frac=0.05,
                                zero_frac=0.002).astype(np.float64)
        f = x.reshape(-1)
        idx = rng.choice(f.size, 6, replace=False)
        f[idx[:3]] = np.sign(f[idx[:3]] + 1e-30) * 2.0 ** -124
        f[idx[3:]] = np.sign(f[idx[3:]] + 1e-30) * 2.0 ** 125
        model = None if name.endswith("lorenzo") else random_model(3, 16, 14)
        return x.astype(np.float32), 5e-7, 8, model, name.endswith("indep")
    if name.startswith("pencil_"):
        # halo-mode pencil decoder edges: one pencil row (n0 < 8), short y,
        # long pencils with a ragged last block, one block column
        shape = {"pencil_thin_z": (3, 17, 40), "pencil_thin_y": (17, 3, 40),
                 "pencil_long": (9, 10, 203), "pencil_single_x": (20, 19, 7)}[name]
        return synth.lognormal_grf(shape, seed=13), 1e-2, 8, random_model(3, 16, 13), False
    if name == "flow_96cubed_B16":
        # block-flow halo decoder (non-pencil shape) with 216 blocks: the size
        # at which a bounded wait of an earlier decoder gave up
        return synth.lognormal_grf((96, 96, 96), seed=15), 1e-2, 16, random_model(3, 16, 15), \
            False
    if name == "flow_B4_1320_blocks":
        return synth.lognormal_grf((48, 40, 44), seed=16), 1e-2, 4, random_model(3, 16, 16), \
            False
    if name.startswith("lanes_"):
        # independent blocks: whole blocks one per lane (several waves, a ragged
        # last wave), clipped blocks one per workgroup
        if name == "lanes_f32_B8":
            return synth.lognormal_grf((72, 64, 136), seed=17), 1e-2, 8, random_model(3, 16, 17), \
                True
        if name == "lanes_B4_ragged":
            return synth.lognormal_grf((30, 41, 53), seed=18), 1e-2, 4, random_model(3, 8, 18), \
                True
        if name == "lanes_2d_B16":
            return synth.zonal_bands_2d((150, 301), seed=19), 1e-2, 16, random_model(2, 32, 19), \
                True
        if name == "lanes_f64":
            x = synth.lognormal_grf((24, 40, 50), seed=20, decades=12, neg_frac=0.1,
                                    zero_frac=0.01, dtype=np.float64)
            return x, 1e-4, 8, random_model(3, 16, 20), True
        if name == "lanes_lorenzo":
            return synth.lognormal_grf((40, 48, 64), seed=22), 1e-2, 8, None, True
    if name == "lorenzo_only":
        return synth.lognormal_grf((30, 31, 66), seed=10), 1e-2, 8, None, False
    if name == "single_point":
        return np.array([[[-2.5]]], dtype=np.float32), 1e-2, 8, random_model(3, 16, 1), False
    if name == "all_zero":
        return np.zeros((9, 10, 11), dtype=np.float32), 1e-2, 8, random_model(3, 16, 1), False
    if name == "tiny_1d":
        return np.array([3.0], dtype=np.float64), 0.5, 2, random_model(1, 4, 1), False
    if name == "sign_gap_delta":  # FP64 rounding closes the sign gap: delta = 1
        x = np.array([1.0, 1.1609689553699987, -1.0, -1.1609689553699987, 1.05, -1.1] * 7,
                     dtype=np.float64).reshape(6, 7)
        return x, 1e-2, 4, random_model(2, 8, 3), False
    raise KeyError(name)


CASES = ["config0_bumps64", "grf_ragged_1e-3", "grf_ragged_indep", "grf_B4_H32", "grf_B16_H8",
         "grf_B5", "zonal_2d", "grf_2d_B64", "grf_1d_halo", "grf_1d_indep", "f64_1e-4",
         "lorenzo_only", "single_point", "all_zero", "tiny_1d", "sign_gap_delta",
         "f32_range_ends_1e-2", "f32_smooth_range_hi", "f32_smooth_range_lo",
         "wide_span_halo", "wide_span_indep", "wide_span_lorenzo",
         "pencil_thin_z", "pencil_thin_y", "pencil_long", "pencil_single_x",
         "flow_96cubed_B16", "flow_B4_1320_blocks", "lanes_f32_B8", "lanes_B4_ragged",
         "lanes_2d_B16", "lanes_f64", "lanes_lorenzo"]


@pytest.mark.parametrize("name", CASES)
def test_codec_bit_exact_vs_oracle(ctx, name):
    x, eps, B, model, indep = _case(name)
    use_net = model is not None
    mode = O.MODE_PLAIN if use_net else O.MODE_LORENZO
    stream = ctx.compress(dev(x), eps, B, model, use_net=use_net, independent=indep)
    g = host_sections(stream)
    if name.startswith("wide_span"):
        assert g["h"]["p_max"] - g["h"]["p_zero"] >= 2 ** 27
    ref = O.compress(x, eps, B, model, mode, independent=indep)
    for k in CONST_KEYS:
        assert g["h"][k] == ref["consts"][k], k
    assert np.array_equal(g["codes"], ref["codes"])
    assert np.array_equal(g["counts"], ref["counts"])
    assert np.array_equal(g["raw"].view(np.uint8), ref["raw"].view(np.uint8))
    xh = ctx.decompress(stream).cpu().numpy()
    ref_xh, _ = O.decompress(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, B, model,
                             mode, independent=indep)
    assert np.array_equal(xh.view(np.uint8), ref_xh.view(np.uint8))
    assert_bound(x, xh, eps)


@pytest.mark.parametrize("shape", [(37, 45, 51), (24, 16, 40)])
def test_decode_output_alignment(ctx, shape):
    """The FP32 inverse writes four values per 16-byte store when the output is
    16-byte aligned and one value per store otherwise; both forms (and the
    ragged tail of n % 4 values) give the same bytes as the oracle, balance
    points included (eps 1e-4 makes some)."""
    x = synth.lognormal_grf(shape, seed=11, decades=10, neg_frac=0.1, zero_frac=0.01)
    eps, B = 1e-4, 8
    stream = ctx.compress(dev(x), eps, B, None, use_net=False)
    ref = O.compress(x, eps, B, None, O.MODE_LORENZO)
    assert len(ref["raw"]) > 0
    ref_xh, _ = O.decompress(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, B, None,
                             O.MODE_LORENZO)
    n = x.size
    buf = torch.full((n + 8,), float("nan"), dtype=torch.float32, device="cuda")
    for off in (0, 1, 2, 3):
        out = buf[off:off + n].view(shape)
        assert (out.data_ptr() % 16 == 0) == (off == 0)
        got = ctx.decompress(stream, out=out).cpu().numpy()
        assert np.array_equal(got.view(np.uint8), ref_xh.view(np.uint8)), off


@pytest.mark.parametrize("shape", [(37, 45, 51), (24, 16, 40)])
def test_compress_input_alignment(ctx, shape):
    """Statistics and grid values read four values per 16-byte load when the
    field is 16-byte aligned and one value per load otherwise; both forms
    (and the ragged tail of n % 4 values) give the same stream."""
    x = synth.lognormal_grf(shape, seed=12, decades=10, neg_frac=0.1, zero_frac=0.01)
    n = x.size
    buf = torch.zeros(n + 8, dtype=torch.float32, device="cuda")
    model = random_model(3, 16, 12)
    ref = None
    for off in (0, 1, 2, 3):
        src = buf[off:off + n].view(shape)
        src.copy_(dev(x))
        assert (src.data_ptr() % 16 == 0) == (off == 0)
        for use_net in (False, True):
            s = ctx.compress(src, 1e-3, 8, model if use_net else None, use_net=use_net).clone()
            if off == 0:
                if not use_net:
                    ref = s
                    o = O.compress(x, 1e-3, 8, None, O.MODE_LORENZO)
                    assert np.array_equal(host_sections(s)["codes"], o["codes"])
                continue
            base = ctx.compress(dev(x), 1e-3, 8, model if use_net else None, use_net=use_net)
            assert torch.equal(s, base), (off, use_net)
    assert ref is not None


def test_determinism_and_histogram(ctx):
    x, eps, B, model, _ = _case("grf_ragged_1e-3")
    a = ctx.compress(dev(x), eps, B, model).clone()
    b = ctx.compress(dev(x), eps, B, model)
    assert torch.equal(a, b)
    hist = ctx.histogram(pwrel.sections(a)["codes"])
    codes = host_sections(a)["codes"]
    assert np.array_equal(hist, np.bincount(codes, minlength=65536).astype(np.uint64))


# --- error paths ----------------------------------------------------------------------------

def test_error_paths(ctx):
    x = synth.lognormal_grf((20, 20, 20), seed=1)
    bad = x.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress(dev(bad), 1e-2, 8, None, use_net=False)
    assert e.value.status == pwrel.ENONFINITE
    out = torch.empty(600, dtype=torch.uint8, device="cuda")
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress(dev(x), 1e-2, 8, None, use_net=False, out=out)
    assert e.value.status == pwrel.ENOSPC
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress(dev(np.array([1e-300, 1e300])), 1e-9, 2, None, use_net=False)
    assert e.value.status == pwrel.ERANGE
    s = ctx.compress(dev(x), 1e-2, 8, None, use_net=False).clone()
    s[0] ^= 0xFF
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.decompress(s, x.shape, torch.float32)
    assert e.value.status == pwrel.ECORRUPT
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.decompress(ctx.compress(dev(x), 1e-2, 8, None, use_net=False)[:-4], x.shape,
                       torch.float32)
    assert e.value.status == pwrel.ECORRUPT
    # an output tensor gives the shape and dtype; the library checks them against the header
    good = ctx.compress(dev(x), 1e-2, 8, None, use_net=False).clone()
    for wrong in (torch.empty((20, 20, 21), dtype=torch.float32, device="cuda"),
                  torch.empty((20, 20, 20), dtype=torch.float64, device="cuda")):
        with pytest.raises(pwrel.PwrelError) as e:
            ctx.decompress(good, out=wrong)
        assert e.value.status == pwrel.EINVAL
    right = torch.empty((20, 20, 20), dtype=torch.float32, device="cuda")
    assert torch.equal(ctx.decompress(good, out=right), ctx.decompress(good))


# --- full size (512^3 FP32), sampled parity and whole-field invariants ------------------------

def stream_to_field_index(shape, B, pos):
    """C-order index of stream positions (block-major order), numpy."""
    n = np.array(shape, dtype=np.int64)
    nb = -(-n // B)
    ext = [np.minimum(B, n[d] - np.arange(nb[d]) * B) for d in range(3)]
    sizes = (ext[0][:, None, None] * ext[1][None, :, None] * ext[2][None, None, :]).ravel()
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    b = np.searchsorted(starts, pos, side="right") - 1
    loc = pos - starts[b]
    bz, by, bx = np.unravel_index(b, tuple(nb))
    ey, ex = ext[1][by], ext[2][bx]
    lx = loc % ex
    ly = (loc // ex) % ey
    lz = loc // (ex * ey)
    return ((bz * B + lz) * n[1] + by * B + ly) * n[2] + bx * B + lx


@pytest.fixture(scope="module")
def big_field():
    return synth.lognormal_grf((512, 512, 512), seed=1001)


@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_full_size_512cubed(ctx, big_field, eps):
    x = big_field
    model = random_model(3, 16, 1001, scale=0.05)
    xd = dev(x)
    stream = ctx.compress(xd, eps, 8, model)
    h = pwrel.header(stream)
    c = O.consts(x, eps)
    for k in CONST_KEYS:
        assert h[k] == c[k], k
    sec = pwrel.sections(stream)
    codes = sec["codes"].cpu().numpy().view(np.uint16)
    counts = sec["counts"].cpu().numpy().view(np.uint32)
    raw = sec["raw"].cpu().numpy()
    # sampled codes against the oracle, point by point
    rng = np.random.default_rng(int(eps * 1e6))
    idx = np.concatenate([rng.choice(x.size, 200000, replace=False),
                          np.arange(0, 512 * 512 * 2),                # first planes (faces)
                          np.arange(x.size - 4096, x.size)])
    ref = O.codes_at(x, c, 8, idx, model, O.MODE_PLAIN)
    assert np.array_equal(codes[ref["pos"].astype(np.int64)], ref["codes"])
    # every balance point: count per block and raw value, in stream order
    zpos = np.flatnonzero(codes == 0)
    assert counts.sum() == zpos.size == h["n_raw"]
    fi = stream_to_field_index(x.shape, 8, zpos)
    assert np.array_equal(raw.view(np.uint32), x.reshape(-1)[fi].view(np.uint32))
    # reconstruction: bound on every point, sampled values bit-exact vs the oracle
    xh = ctx.decompress(stream)
    hd, xt = xh.double(), xd.double()
    z = xt == 0
    assert bool(torch.all(hd[z] == 0))
    assert bool(torch.all(torch.signbit(hd[~z]) == torch.signbit(xt[~z])))
    assert bool(torch.all((xt - hd).abs() <= eps * xt.abs()))
    xh_s = xh.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref_xh = O.inverse_field(ref["p"], c, np.float32)
    is_raw = ref["codes"] == 0
    ref_xh[is_raw] = x.reshape(-1)[idx[is_raw]]
    assert np.array_equal(xh_s.view(np.uint32), ref_xh.view(np.uint32))


# --- FP32 fast paths ------------------------------------------------------------------------

def test_fastmath_bounds_hold(ctx):
    """The hardware log2 / exp2 errors, over every input the fast paths can
    receive, stay within the bounds the kernels assume."""
    lerr, eerr = ctx.fastmath_check()
    assert 0.0 < lerr <= pwrel.FAST_LOG2_ERR, lerr
    assert 0.0 < eerr <= pwrel.FAST_EXP2_ERR, eerr


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_fast_path_boundaries(ctx, eps):
    """Values swept densely across grid cells (both rounding boundaries of the
    transform and both ends of the bound check, both signs): codes, counts and
    raw values bit-exact to the oracle's FP64 path."""
    anchors = np.array([1e-3, 1e3, -1e-3, -1e3, 0.0], dtype=np.float32)
    c = O.consts(anchors, eps)
    rng = np.random.default_rng(11)
    lo, hi = int(c["p_zero"]) + 2, int(c["b_sign"]) - 2
    cells = rng.integers(lo, hi, 120)
    ncell = int(c["n_lo"]) + 2 + rng.integers(0, hi - lo, 120)
    p = np.concatenate([cells, ncell]).astype(np.int32)
    centre = O.inverse_field(p, c, np.float32).astype(np.float64)
    s = np.linspace(-1.25, 1.25, 1001) * c["b_a"]
    x = (centre[:, None] * np.exp2(s)[None, :]).astype(np.float32).ravel()
    x = x[(np.abs(x) > 1e-3) & (np.abs(x) < 1e3)]
    # neighbours in the float grid of a few sweep points: every ulp near the edges
    edge = x[::97]
    ulps = np.concatenate([np.nextafter(edge, np.float32(np.inf)),
                           np.nextafter(edge, np.float32(-np.inf))]).astype(np.float32)
    x = np.concatenate([anchors, x, ulps]).astype(np.float32)
    n = (x.size // 64) * 64
    x = np.ascontiguousarray(np.concatenate([anchors, x[5:n]]).reshape(-1, 64))
    assert O.consts(x, eps)["Lp"] == c["Lp"]
    stream = ctx.compress(dev(x), eps, 8, None, use_net=False)
    g = host_sections(stream)
    ref = O.compress(x, eps, 8, None, O.MODE_LORENZO)
    assert np.array_equal(g["codes"], ref["codes"])
    assert np.array_equal(g["counts"], ref["counts"])
    assert np.array_equal(g["raw"].view(np.uint8), ref["raw"].view(np.uint8))
    xh = ctx.decompress(stream).cpu().numpy()
    assert_bound(x, xh, eps)
    # the sweep reaches both verdicts of the bound check
    assert 0 < g["h"]["n_raw"] < x.size


# --- sections in separate buffers (pwrel_compress_raw) and the stored network -----------------

@pytest.mark.parametrize("judge", [False, True])
def test_compress_raw_equals_stream_sections(ctx, judge):
    x = synth.lognormal_grf((37, 45, 51), seed=21, decades=10, neg_frac=0.1, zero_frac=0.01)
    model = random_model(3, 16, 21)
    xd = dev(x)
    stream = ctx.compress(xd, 1e-3, 8, model, judge=judge)
    sec = pwrel.sections(stream)
    r = ctx.compress_raw(xd, 1e-3, 8, model, judge=judge)
    h, hr = sec["header"], r["header"]
    assert h["n_raw"] > 0
    for k in h:
        assert hr[k] == h[k], k
    assert torch.equal(r["codes"], sec["codes"])
    assert torch.equal(r["counts"], sec["counts"])
    assert torch.equal(r["raw"], sec["raw"])
    if judge:
        assert torch.equal(r["bflags"], sec["bflags"])
    # too small a raw capacity is reported, not overrun
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_raw(xd, 1e-3, 8, model, judge=judge, raw_capacity=h["n_raw"] - 1)
    assert e.value.status == pwrel.ENOSPC


def test_stream_model_and_saved_model_compress_alike(ctx):
    x = synth.lognormal_grf((40, 40, 48), seed=22)
    model, _ = ctx.train(dev(x), 1e-2, 8, rho=0.05, seed=22, hidden=16, precision=1)
    a = ctx.compress(dev(x), 1e-2, 8, model, judge=True).clone()
    kept = pwrel.model_load(pwrel.model_save(ctx.stream_model(a)))
    b = ctx.compress(dev(x), 1e-2, 8, kept, judge=True)
    assert torch.equal(a, b)
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.stream_model(ctx.compress(dev(x), 1e-2, 8, None, use_net=False))
    assert e.value.status == pwrel.EINVAL


def test_unaligned_stream_buffers_are_refused(ctx):
    """Stream buffers must start 16-byte aligned (the kernels move them in
    16-byte vectors and update shared words atomically): an output or a stream
    starting one byte in is refused before any GPU work, by every entry point
    that writes or reads a stream."""
    x = dev(synth.lognormal_grf((16, 16, 16), seed=41))
    cap = pwrel.compress_bound(tuple(x.shape), pwrel.F32, 8)
    buf = torch.empty(cap + 16, dtype=torch.uint8, device="cuda")
    for fn in (ctx.compress, ctx.compress_noalloc):
        with pytest.raises(pwrel.PwrelError) as e:
            fn(x, 1e-2, 8, None, use_net=False, out=buf[1:1 + cap])
        assert e.value.status == pwrel.EINVAL
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_batch([x], 1e-2, use_net=False, outs=[buf[1:1 + cap]])
    assert e.value.status == pwrel.EINVAL
    s = ctx.compress(x, 1e-2, 8, None, use_net=False)
    moved = torch.empty(s.numel() + 16, dtype=torch.uint8, device="cuda")
    moved[1:1 + s.numel()].copy_(s)
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.decompress(moved[1:1 + s.numel()], shape=tuple(x.shape), dtype=torch.float32)
    assert e.value.status == pwrel.EINVAL
    # the same bytes at an aligned address decode
    xh = ctx.decompress(moved[1:1 + s.numel()].clone())
    assert xh.shape == x.shape
