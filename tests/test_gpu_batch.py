"""Batched compression (pwrel_compress_batch) against single-field compression.

Each field's stream from the batched launches must be byte-identical to the
stream pwrel_compress writes for that field alone (same bound, block, model
and options); single-field streams are themselves held bit-exact to the
oracle by the codec tests, and a sample of fields is checked against the
oracle here too.  Covers 2-D and 3-D fields of uneven, ragged shapes in one
call, Lorenzo-only, FP32 and BF16 networks, the judge, independent blocks, a
field that fails (NaN) next to fields that do not, argument errors, a
repeated request on another stream, and a HIP graph captured from a repeated
request and replayed over changing inputs.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth

pytestmark = pytest.mark.gpu

SHAPES = [(37, 45, 51), (8, 8, 8), (1, 1, 1), (3, 70, 9), (40, 17, 66), (150, 301), (16, 16),
          (5, 300), (1, 1), (64, 129), (33, 65, 130), (257, 31)]


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


def fields(seed0=0, shapes=SHAPES):
    xs = []
    for i, s in enumerate(shapes):
        x = synth.lognormal_grf(s, seed=seed0 + 17 * i, decades=6, neg_frac=0.05,
                                zero_frac=0.005)
        xs.append(torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda())
    return xs


def model(ndim, H, seed, precision=0):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, 0.2, size=(H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 0.5, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.2, H)).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal(0, 0.3)))
    m["precision"] = precision
    return m


def single(ctx, xs, eps, models, **kw):
    out = []
    for x in xs:
        B = 8 if x.dim() == 3 else 16
        m = models.get(x.dim()) if models else None
        s = ctx.compress(x, eps, block=B, model=m, use_net=m is not None, **kw)
        out.append(s.cpu().numpy().copy())
    return out


CASES = {
    "lorenzo": dict(eps=1e-2, models=None, judge=False, independent=False),
    "net_fp32": dict(eps=1e-3, models={2: ("m", 2, 16, 1, 0), 3: ("m", 3, 16, 2, 0)},
                     judge=False, independent=False),
    "bf16_judge": dict(eps=1e-2, models={2: ("m", 2, 32, 3, 1), 3: ("m", 3, 32, 4, 1)},
                       judge=True, independent=False),
    "fp32_judge_indep": dict(eps=1e-2, models={2: ("m", 2, 8, 5, 0), 3: ("m", 3, 8, 6, 0)},
                             judge=True, independent=True),
}


def make_models(spec):
    if spec is None:
        return None
    return {nd: model(a, H, seed, prec) for nd, (_, a, H, seed, prec) in spec.items()}


@pytest.mark.parametrize("case", list(CASES))
def test_batch_matches_single(ctx, case):
    c = CASES[case]
    print(f"batch case {case}", flush=True)
    xs = fields(seed0=100)
    models = make_models(c["models"])
    kw = dict(judge=c["judge"], independent=c["independent"])
    got = ctx.compress_batch(xs, c["eps"], models=models, use_net=models is not None, **kw)
    want = single(ctx, xs, c["eps"], models, **kw)
    for i, (g, w) in enumerate(zip(got, want)):
        g = g.cpu().numpy()
        assert g.size == w.size, (case, i, SHAPES[i])
        assert np.array_equal(g, w), (case, i, SHAPES[i])


def test_batch_oracle_sample(ctx):
    """Fields of a batch held to the oracle directly: codes, counts, raw
    values and the decoded field, bit for bit."""
    print("batch oracle sample", flush=True)
    xs = fields(seed0=7)
    eps = 1e-2
    got = ctx.compress_batch(xs, eps, use_net=False)
    for i in (0, 4, 5, 11):
        x = xs[i].cpu().numpy()
        B = 8 if x.ndim == 3 else 16
        ref = O.compress(x, eps, B, None, O.MODE_LORENZO)
        sec = pwrel.sections(got[i])
        assert np.array_equal(sec["codes"].cpu().numpy().view(np.uint16), ref["codes"]), i
        assert np.array_equal(sec["counts"].cpu().numpy().view(np.uint32), ref["counts"]), i
        assert np.array_equal(sec["raw"].cpu().numpy().view(np.uint8), ref["raw"].view(np.uint8)), i
        xh = ctx.decompress(got[i]).cpu().numpy()
        ref_xh, _ = O.decompress(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, B,
                                 None, O.MODE_LORENZO)
        assert np.array_equal(xh.view(np.uint8), ref_xh.view(np.uint8)), i


def test_batch_failed_field(ctx):
    """A field with a NaN fails alone: size 0, status in its header; the
    other fields' streams are unaffected."""
    print("batch failed field", flush=True)
    xs = fields(seed0=300, shapes=[(20, 20, 20), (50, 60), (9, 10, 11)])
    xs[1][3, 4] = float("nan")
    outs, sizes = ctx.compress_batch(xs, 1e-2, use_net=False, views=False)
    torch.cuda.synchronize()
    sz = sizes.cpu().tolist()
    assert sz[1] == 0
    raw = outs[1][:pwrel.C.sizeof(pwrel.Header)].cpu().numpy().tobytes()
    assert pwrel.Header.from_buffer_copy(raw).status == pwrel.ENONFINITE
    want = single(ctx, [xs[0], xs[2]], 1e-2, None)
    for i, w in zip((0, 2), want):
        assert sz[i] == w.size
        assert np.array_equal(outs[i][:sz[i]].cpu().numpy(), w)


def test_batch_argument_errors(ctx):
    print("batch argument errors", flush=True)
    x3 = fields(shapes=[(10, 10, 10)])[0]
    x1 = torch.ones(100, device="cuda")
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_batch([x3, x1], 1e-2, use_net=False)
    assert e.value.status == pwrel.EINVAL
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_batch([x3], 1e-2, use_net=False, blocks={3: 4})
    assert e.value.status == pwrel.EINVAL
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_batch([x3], 1e-2, use_net=True, models={})
    assert e.value.status == pwrel.EINVAL
    small = [torch.empty(64, dtype=torch.uint8, device="cuda")]
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_batch([x3], 1e-2, use_net=False, outs=small)
    assert e.value.status == pwrel.ENOSPC
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_batch([x3.double()], 1e-2, use_net=False)
    assert e.value.status == pwrel.EINVAL


def test_batch_repeat_other_stream(ctx):
    print("batch repeat on another stream", flush=True)
    xs = fields(seed0=500)
    outs, sizes = ctx.compress_batch(xs, 1e-2, use_net=False, views=False)
    torch.cuda.synchronize()
    first = [o[:s].cpu().numpy().copy() for o, s in zip(outs, sizes.cpu().tolist())]
    for o in outs:
        o.zero_()
    sizes.zero_()
    torch.cuda.synchronize()
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        ctx.compress_batch(xs, 1e-2, use_net=False, outs=outs, sizes=sizes, views=False,
                           stream=s2)
    s2.synchronize()
    for o, s, f in zip(outs, sizes.cpu().tolist(), first):
        assert np.array_equal(o[:s].cpu().numpy(), f)


def test_batch_graph_replay(ctx):
    """A repeated request captured in a HIP graph, replayed over new inputs
    (copied into the same tensors), with eager work between the replays."""
    print("batch graph replay", flush=True)
    models = make_models(CASES["bf16_judge"]["models"])
    xs = fields(seed0=900)
    outs, sizes = ctx.compress_batch(xs, 1e-2, models=models, judge=True, views=False)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ctx.compress_batch(xs, 1e-2, models=models, judge=True, outs=outs, sizes=sizes,
                               views=False, stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        new = fields(seed0=1000 + 31 * rep)
        for x, n in zip(xs, new):
            x.copy_(n)
        for o in outs:
            o.fill_(0xAB)
        sizes.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = single(ctx, new, 1e-2, models, judge=True)
        sz = sizes.cpu().tolist()
        for i, w in enumerate(want):
            assert sz[i] == w.size, (rep, i)
            assert np.array_equal(outs[i][:sz[i]].cpu().numpy(), w), (rep, i)


def test_batch_tile_variants_and_tuner(ctx):
    """Every tile shape variant writes the same streams; the tuner keeps a
    valid variant per class and leaves the request's outputs written."""
    print("batch tile variants", flush=True)
    models = make_models(CASES["bf16_judge"]["models"])
    xs = fields(seed0=1300)
    want = single(ctx, xs, 1e-2, models, judge=True)
    try:
        for v in range(pwrel.BATCH_TILES):
            var, shapes = ctx.batch_tiles([v, v])
            assert var == [v, v]
            got = ctx.compress_batch(xs, 1e-2, models=models, judge=True)
            for i, w in enumerate(want):
                assert np.array_equal(got[i].cpu().numpy(), w), (v, i, shapes)
        with pytest.raises(pwrel.PwrelError):
            ctx.batch_tiles([pwrel.BATCH_TILES, 0])
        req = ctx.batch_request(xs, 1e-2, models=models, judge=True)
        var, ms = req.tune(reps=2)
        assert all(0 <= v < pwrel.BATCH_TILES for v in var)
        assert ctx.batch_tiles()[0] == var
        assert all(m > 0 for m in ms[0]) and all(m > 0 for m in ms[1])
        got = req.views()
        for i, w in enumerate(want):
            assert np.array_equal(got[i].cpu().numpy(), w), ("tuned", i)
    finally:
        ctx.batch_tiles([0, 0])
