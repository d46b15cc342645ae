"""Data blocks (Sec. 5: a stream carries factor_pos and factor_neg for its
data block; Algorithm 1 computes them from its input's extreme values).

A field split into sub-volumes of edge `sub`, each compressed into its own
stream with its own factors by one gather and one batched compression:
- every data block's stream is byte for byte the stream pwrel_compress
  writes for that sub-volume alone (Lorenzo, FP32 network with the judge,
  BF16 network; clipped data blocks at the high faces);
- the data blocks' factors are the oracle's constants of each sub-volume,
  and the codes, counts and raw values of a sample are the oracle's;
- the round trip puts every sub-volume back: equal to decoding each stream
  alone, and within the bound on every point;
- bad arguments are refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth
from tests.test_gpu_codec import assert_bound, dev, random_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def field():
    return synth.lognormal_grf((70, 90, 100), seed=61, decades=8, neg_frac=0.1, zero_frac=0.01)


def sub_views(x, sub):
    n = x.shape
    for bz in range(0, n[0], sub):
        for by in range(0, n[1], sub):
            for bx in range(0, n[2], sub):
                yield x[bz:bz + sub, by:by + sub, bx:bx + sub]


CASES = {"lorenzo": (None, False, False), "fp32_judge_indep": ((3, 16, 62, 0), True, True),
         "bf16": ((3, 32, 63, 1), False, False)}


@pytest.mark.parametrize("case", list(CASES))
def test_datablocks_equal_single_streams(ctx, field, case):
    spec, judge, indep = CASES[case]
    model = None
    if spec:
        model = random_model(*spec[:3])
        model["precision"] = spec[3]
    print(f"[datablocks] {case}", flush=True)
    xd = dev(field)
    outs, sizes = ctx.compress_datablocks(xd, 1e-2, 32, model, use_net=model is not None,
                                          judge=judge, independent=indep)
    sz = sizes.cpu().tolist()
    views = list(sub_views(xd, 32))
    assert len(views) == outs.shape[0] == 3 * 3 * 4
    for i, v in enumerate(views):
        single = ctx.compress(v.contiguous(), 1e-2, 8, model, use_net=model is not None,
                              judge=judge, independent=indep)
        assert sz[i] == single.numel(), i
        assert torch.equal(outs[i, :sz[i]], single), i


def test_datablocks_factors_match_oracle(ctx, field):
    xd = dev(field)
    outs, sizes = ctx.compress_datablocks(xd, 1e-2, 32, None, use_net=False)
    sz = sizes.cpu().tolist()
    lps = set()
    for i, v in enumerate(sub_views(field, 32)):
        v = np.ascontiguousarray(v)
        h = pwrel.header(outs[i, :sz[i]])
        c = O.consts(v, 1e-2)
        assert h["Lp"] == c["Lp"] and h["Ln"] == c["Ln"], i
        assert h["p_zero"] == c["p_zero"] and h["b_sign"] == c["b_sign"], i
        lps.add(h["Lp"])
        if i % 7 == 0:  # a sample against the oracle's codec
            ref = O.compress(v, 1e-2, 8, None, O.MODE_LORENZO)
            sec = pwrel.sections(outs[i, :sz[i]])
            assert np.array_equal(sec["codes"].cpu().numpy().view(np.uint16), ref["codes"]), i
            assert np.array_equal(sec["counts"].cpu().numpy().view(np.uint32), ref["counts"]), i
            assert np.array_equal(sec["raw"].cpu().numpy().view(np.uint8),
                                  ref["raw"].view(np.uint8)), i
    assert len(lps) > 10  # the data blocks carry factors of their own


def test_datablocks_round_trip(ctx, field):
    xd = dev(field)
    model = random_model(3, 16, 64)
    outs, sizes = ctx.compress_datablocks(xd, 1e-2, 32, model, judge=True, independent=True)
    back = ctx.decompress_datablocks(outs, sizes, tuple(field.shape), 32)
    want = torch.empty_like(xd)
    sz = sizes.cpu().tolist()
    k = 0
    n = field.shape
    for bz in range(0, n[0], 32):
        for by in range(0, n[1], 32):
            for bx in range(0, n[2], 32):
                want[bz:bz + 32, by:by + 32, bx:bx + 32] = ctx.decompress(outs[k, :sz[k]].clone())
                k += 1
    assert torch.equal(back.view(torch.int32), want.view(torch.int32))
    assert_bound(field, back.cpu().numpy(), 1e-2)


def test_datablocks_arguments(ctx, field):
    xd = dev(field)
    for sub in (12, 4, 0):
        with pytest.raises(pwrel.PwrelError) as e:
            ctx.compress_datablocks(xd, 1e-2, sub, None, use_net=False)
        assert e.value.status == pwrel.EINVAL
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.compress_datablocks(xd, 1e-2, 32, None, use_net=False, stride=1000)
    assert e.value.status == pwrel.EINVAL
    outs, sizes = ctx.compress_datablocks(xd, 1e-2, 32, None, use_net=False)
    bad = sizes.cpu().clone()
    bad[3] = outs.shape[1] + 1
    with pytest.raises(pwrel.PwrelError) as e:
        ctx.decompress_datablocks(outs, bad, tuple(field.shape), 32)
    assert e.value.status == pwrel.ECORRUPT
