"""Full-size GPU runs of the two workloads beyond the 512^3 FP32 field:

- the FP64 volume of 1024 x 1024 x 512 values (4 GiB, C-order dims
  (512, 1024, 1024); log-normal k^-3 field over 12 decades, 10 % negative
  connected regions, 1 % zeros) at eps = 1e-4: the FP64 transform and bound
  check on the device, a network in FP32.  Its byte offsets pass 2^32.
  Checked against the FP64 oracle: header constants; codes at 200,000 sampled
  points plus the first and last planes; every balance point's count and raw
  value; the reconstruction of EVERY point equal to the oracle's inverse of
  the oracle's grid value (the oracle run over the field in chunks on the
  host threads), plus bound, sign and zero on every point;
- the 2-D field of 1800 x 3600 values (zonal bands plus k^-2 noise, block
  16^2) on the learned path: network of width 32 trained on the device from
  1 % of the points, BF16 matrix-core inference, per-block judge.  Checked:
  Lorenzo blocks' codes equal the oracle's at every point; network blocks'
  implied predictions within 1/2 + the derived BF16 bound of the network's
  FP64 value at every full-stencil point; the reconstruction equal to the
  oracle's inverse everywhere (raw values at balance points); bound, sign,
  zero everywhere.
"""
import concurrent.futures as cf

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2309_09778_amd import pwrel, synth

pytestmark = pytest.mark.gpu

R = 32768
CONST_KEYS = ("eps0", "b_a", "w", "r", "Lp", "Ln", "d0", "p_zero", "b_sign", "n_lo", "delta")


@pytest.fixture(scope="module")
def ctx():
    c = pwrel.Context(0)
    yield c
    c.close()


def chunked(fn, n, parts=16):
    """Run fn(lo, hi) over [0, n) in parts on host threads (the oracle's C
    routines release the interpreter lock)."""
    step = -(-n // parts)
    with cf.ThreadPoolExecutor(parts) as ex:
        list(ex.map(lambda lo: fn(lo, min(n, lo + step)), range(0, n, step)))


def oracle_reconstruction(x_flat, c, dtype):
    """The oracle's x^ of every point by R1: the inverse of its grid value."""
    n = x_flat.size
    out = np.empty(n, dtype=dtype)

    def part(lo, hi):
        p = O.transform_field(x_flat[lo:hi], c)
        out[lo:hi] = O.inverse_field(p, c, dtype)
    chunked(part, n)
    return out


def assert_bound_device(xd, xh, eps):
    hd, xt = xh.double(), xd.double()
    z = xt == 0
    assert bool(torch.all(hd[z] == 0))
    assert bool(torch.all(torch.signbit(hd[~z]) == torch.signbit(xt[~z])))
    assert bool(torch.all((xt - hd).abs() <= eps * xt.abs()))


def fp32_model(ndim, H, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    K = (1 << ndim) - 2
    m = O.mlp_init(ndim, H, seed=seed)
    m["w1"] = (m["w1"] + rng.normal(0, scale, size=(H, K))).astype(np.float32)
    m["v"] = (m["v"] + rng.normal(0, scale, H)).astype(np.float32)
    return m


def test_fp64_volume_4gib(ctx):
    shape, eps, B = (512, 1024, 1024), 1e-4, 8
    print(f"[full] FP64 {shape} eps {eps}: generating", flush=True)
    xd = synth.lognormal_grf_device(shape, seed=1004, decades=12, neg_frac=0.10, zero_frac=0.01,
                                    dtype=torch.float64)
    assert xd.numel() * 8 == 4 << 30  # byte offsets into the field pass 2^32
    model = fp32_model(3, 16, 1004)
    stream = ctx.compress(xd, eps, B, model)
    assert stream.numel() > (1 << 30)  # the codes alone are 1 GiB
    xh = ctx.decompress(stream)
    torch.cuda.synchronize()
    print("[full] FP64 compressed and decompressed", flush=True)
    assert_bound_device(xd, xh, eps)
    x = xd.cpu().numpy()
    h = pwrel.header(stream)
    c = O.consts(x, eps)
    for k in CONST_KEYS:
        assert h[k] == c[k], k
    sec = pwrel.sections(stream)
    codes = sec["codes"].cpu().numpy().view(np.uint16)
    counts = sec["counts"].cpu().numpy().view(np.uint32)
    raw = sec["raw"].cpu().numpy()
    # a rough 12-decade field at eps = 1e-4: prediction errors beyond the 2^15 code range are
    # common, so many values are balance points (stored raw)
    print(f"[full] FP64 balance points: {h['n_raw']} of {x.size}", flush=True)
    assert 0 < h["n_raw"] < x.size
    # sampled codes (random points, the first two planes, the last points)
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(x.size, 200000, replace=False),
                          np.arange(0, 2 * 1024 * 1024, 7), np.arange(x.size - 8192, x.size)])
    ref = O.codes_at(x, c, B, idx, model, O.MODE_PLAIN)
    assert np.array_equal(codes[ref["pos"].astype(np.int64)], ref["codes"])
    # every balance point: per-block counts, raw values in stream order
    zpos = np.flatnonzero(codes == 0)
    assert counts.sum() == zpos.size == h["n_raw"]
    nb = [s // B for s in shape]
    blk, loc = zpos // 512, zpos % 512
    bz, by, bx = blk // (nb[1] * nb[2]), (blk // nb[2]) % nb[1], blk % nb[2]
    lz, ly, lx = loc // 64, (loc // 8) % 8, loc % 8
    fi = ((bz * 8 + lz) * shape[1] + by * 8 + ly) * shape[2] + bx * 8 + lx
    assert np.array_equal(raw.view(np.uint64), x.reshape(-1)[fi].view(np.uint64))
    # the reconstruction of every point against the oracle
    print("[full] FP64 oracle reconstruction of every point", flush=True)
    xr = oracle_reconstruction(x.reshape(-1), c, np.float64)
    xr[fi] = x.reshape(-1)[fi]
    assert np.array_equal(xh.cpu().numpy().reshape(-1).view(np.uint64), xr.view(np.uint64))


def test_zonal_2d_learned_full_size(ctx):
    shape, eps, B = (1800, 3600), 1e-2, 16
    x = synth.zonal_bands_2d(shape, seed=1002)
    xd = torch.from_numpy(x).cuda()
    model, rep = ctx.train(xd, eps, B, rho=0.01, seed=1002, hidden=32, precision=1)
    print(f"[full] 2-D trained: chosen {rep['chosen']}, {rep['n_train']} pairs", flush=True)
    stream = ctx.compress(xd, eps, B, model, judge=True)
    xh = ctx.decompress(stream)
    assert_bound_device(xd, xh, eps)
    sec = pwrel.sections(stream)
    codes_s = sec["codes"].cpu().numpy().view(np.uint16)
    flags = sec["bflags"].cpu().numpy()
    c = O.consts(x, eps)
    # stream position of every field point: block rows of height hb = min(B, 1800 - by*B)
    # (the last one is ragged), blocks of width B (3600 = 225 * 16), local raster order
    nby, nbx = -(-shape[0] // B), -(-shape[1] // B)
    yy, xx = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    by, bx = yy // B, xx // B
    hb = np.minimum(B, shape[0] - by * B)
    bw = np.minimum(B, shape[1] - bx * B)
    pos = by * B * shape[1] + bx * B * hb + (yy % B) * bw + (xx % B)
    assert np.array_equal(np.sort(pos.reshape(-1)), np.arange(x.size))
    codes = codes_s[pos]
    lor = O.compress(x, eps, B, None, O.MODE_LORENZO)
    lcodes = lor["codes"][pos]
    bflag = flags[by * nbx + bx].astype(bool)
    assert 0 < flags.mean() < 1
    assert np.array_equal(codes[~bflag], lcodes[~bflag])
    p = lor["p"]
    full = np.zeros(shape, dtype=bool)
    full[1:, 1:] = True
    face = bflag & ~full
    assert np.array_equal(codes[face], lcodes[face])
    sel = bflag & full
    n1 = np.zeros_like(p)
    n1[:, 1:] = p[:, :-1]
    # inputs of the 2-D network: u_0 = n_2 - n_1 (row above), u_1 = n_3 - n_1 (above-left)
    up = np.zeros_like(p)
    up[1:, :] = p[:-1, :]
    ul = np.zeros_like(p)
    ul[1:, 1:] = p[:-1, :-1]
    u = np.stack([up - n1, ul - n1], -1)[sel].astype(np.float32)
    y64, bound = O.mlp_eval_f64(model, u)
    cg = codes[sel].astype(np.int64)
    coded = cg != 0
    y_int = cg - R + p[sel].astype(np.int64) - n1[sel].astype(np.int64)
    d = np.abs(y_int[coded] - y64[coded])
    assert np.all(d <= 0.5 + bound[coded]), (d - bound[coded]).max()
    # reconstruction of every point
    xr = O.inverse_field(p, c, np.float32)
    zr = codes == 0
    xr[zr] = x[zr]
    assert np.array_equal(xh.cpu().numpy().view(np.uint32), xr.view(np.uint32))
