"""GPU open-loop mode (the paper's literal prediction from raw neighbours,
Sec. 4.3, 4.4.1, 4.4.2) against the oracle's open-loop mode: codes, per-block
counts, raw values and the decoder's reconstruction bit for bit, the
coverage histogram, the chosen m, and the reported violations and largest
relative error; on ragged 1-D / 2-D / 3-D fields, FP32 and FP64, Lorenzo and
the FP32 network, fixed and coverage-chosen m, with and without deliberate
balance points."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


def model(ndim, H, seed):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, 0.05, size=(H, K))).astype(np.float32)
    m["b1"] = rng.normal(0, 0.1, H).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.05, H)).astype(np.float32)
    m["b2"] = float(np.float32(rng.normal(0, 0.1)))
    return m


CASES = {
    "3d_lorenzo": (lambda: synth.lognormal_grf((19, 22, 37), seed=1), 1e-2, 8, None, 16, 0),
    "3d_lorenzo_cov": (lambda: synth.lognormal_grf((19, 22, 37), seed=1), 1e-2, 8, None, 0, 0),
    "3d_net_m8_gap16": (lambda: synth.lognormal_grf((17, 20, 26), seed=2), 1e-2, 8,
                        (3, 16, 3), 8, 16),
    "3d_B4_gap3": (lambda: synth.lognormal_grf((13, 14, 15), seed=3), 1e-3, 4, None, 0, 3),
    "2d_cov": (lambda: synth.zonal_bands_2d((70, 131), seed=4), 2e-2, 16, None, 0, 0),
    "2d_net": (lambda: synth.zonal_bands_2d((70, 131), seed=4), 1e-2, 16, (2, 8, 5), 12, 0),
    "1d": (lambda: synth.lognormal_grf((3001,), seed=6), 1e-2, 64, None, 16, 0),
    "3d_f64": (lambda: synth.lognormal_grf((15, 17, 19), seed=7, dtype=np.float64), 1e-4, 8,
               None, 0, 8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_openloop_bit_exact_vs_oracle(ctx, name):
    make, eps, B, net, mbits, gap = CASES[name]
    print(f"open-loop case {name}", flush=True)
    x = make()
    m = model(*net) if net else None
    r = ctx.openloop(torch.from_numpy(np.ascontiguousarray(x)).cuda(), eps, B, m, mbits, gap)
    rep = r["report"]
    mb = mbits
    if mbits == 0:
        ref0 = O.openloop_encode(x, eps, B, m, 16, gap)
        mb = O.openloop_choose_m(ref0["hist"], eps)
    assert rep["mbits"] == mb
    ref = O.openloop_encode(x, eps, B, m, mb, gap)
    assert rep["hist"] == ref["hist"].tolist()
    assert np.array_equal(r["codes"].cpu().numpy().view(np.uint16), ref["codes"])
    assert np.array_equal(r["counts"].cpu().numpy().view(np.uint32), ref["counts"])
    assert rep["n_raw"] == ref["raw"].size
    assert np.array_equal(r["raw"].cpu().numpy().view(np.uint8), ref["raw"].view(np.uint8))
    xh, _ = O.openloop_decode(ref["codes"], ref["raw"], ref["consts"], x.shape, x.dtype, B, m, mb)
    got = r["xhat"].cpu().numpy()
    assert np.array_equal(got.view(np.uint8), xh.view(np.uint8))
    orep = O.openloop_report(x, xh, eps)
    assert rep["violations"] == orep["violations"]
    assert rep["max_rel_error"] == orep["max_rel"]


def test_openloop_every_point_balanced_reproduces_field(ctx):
    x = synth.lognormal_grf((9, 10, 11), seed=8)
    r = ctx.openloop(torch.from_numpy(x).cuda(), 1e-2, 4, None, 16, 1)
    assert r["report"]["violations"] == 0 and r["report"]["n_raw"] == x.size
    assert np.array_equal(r["xhat"].cpu().numpy().view(np.uint32), x.view(np.uint32))


def test_openloop_argument_errors(ctx):
    x = torch.ones((8, 8, 8), device="cuda")
    for kw in (dict(mbits=1), dict(mbits=17), dict(gap=-1)):
        with pytest.raises(pwrel.PwrelError) as e:
            ctx.openloop(x, 1e-2, 8, **kw)
        assert e.value.status == pwrel.EINVAL
