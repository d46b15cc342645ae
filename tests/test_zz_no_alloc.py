"""pwrel_compress_noalloc (static device scratch, no allocation) against
pwrel_compress: byte-identical streams on two calls in a row, the second on a
smaller field, through the C ABI; the size limit is rejected before any GPU
work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth

pytestmark = pytest.mark.gpu


def _model(ndim, H, seed, precision):
    rng = np.random.default_rng(seed)
    m = O.mlp_init(ndim, H, seed=seed)
    K = (1 << ndim) - 2
    m["w1"] = (m["w1"] + rng.normal(0, 0.1, size=(H, K))).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, 0.1, H)).astype(np.float32)
    m["precision"] = precision
    return m


def test_noalloc_matches_compress_twice():
    ctx = pwrel.Context(0)
    try:
        runs = [((96, 80, 72), np.float32, 8, dict(model=_model(3, 32, 5, 1), judge=True)),
                ((33, 41, 29), np.float32, 8, dict(model=_model(3, 16, 6, 0))),
                ((17, 300), np.float64, 16, dict(model=None, use_net=False))]
        for shape, dt, B, kw in runs:
            print(f"[noalloc] {shape} {np.dtype(dt).name} B={B}", flush=True)
            x = synth.lognormal_grf(shape, seed=len(shape) * 100 + shape[0], decades=8,
                                    neg_frac=0.1, zero_frac=0.005).astype(dt)
            xd = torch.from_numpy(x).cuda()
            ref = ctx.compress(xd, 1e-2, B, **kw).cpu().numpy()
            cap = pwrel.compress_bound(shape, pwrel.F32 if dt == np.float32 else pwrel.F64, B)
            out = torch.full((cap,), 0xAB, dtype=torch.uint8, device="cuda")
            got = ctx.compress_noalloc(xd, 1e-2, B, out=out, **kw).cpu().numpy()
            assert got.size == ref.size
            assert np.array_equal(got, ref)
            # and it decodes to the oracle's reconstruction of the bound
            xh = ctx.decompress(torch.from_numpy(got).cuda()).cpu().numpy()
            nz = x != 0
            assert np.all(xh[~nz] == 0)
            assert np.all(np.abs(x[nz].astype(np.float64) - xh[nz]) <= 1e-2 * np.abs(x[nz]))
    finally:
        ctx.close()


def test_noalloc_rejects_fields_beyond_its_scratch():
    ctx = pwrel.Context(0)
    try:
        xd = torch.ones((1 << 22) + 1, dtype=torch.float32, device="cuda")
        with pytest.raises(pwrel.PwrelError) as ei:
            ctx.compress_noalloc(xd, 1e-2, 256, use_net=False)
        assert ei.value.status == pwrel.EINVAL and "static scratch" in str(ei.value)
    finally:
        ctx.close()
