"""Seeded synthetic fields shaped like the paper's workloads.

The paper evaluates on SEG-Y seismic volumes that are not available here;
these generators stand in for them.  This module holds no part of the
compressor's arithmetic: it only draws numbers.  Both the CPU oracle and the
GPU library are fed from it.

Recipes (seed fixed per call):
  gaussian_bumps  -- 8 Gaussian bumps (centres uniform, widths 4..16 cells,
                     amplitudes log-uniform 1e-3..1e3 with random sign) plus
                     3 unit-amplitude sine modes (integer wave numbers 1..4,
                     random phase), then an exact fraction of voxels set to 0.
  lognormal_grf   -- |x| = 10^(decades/2 * g / max|g|) with g a periodic
                     Gaussian random field of power spectrum k^-slope
                     (standardised), sign negative where an independent field
                     of the same spectrum exceeds its (1 - neg_frac) quantile
                     (connected regions), then an exact fraction of zeros.
  zonal_bands_2d  -- sum_j (1/j) cos(2 pi j (i_lat + 1/2) / n_lat), j = 1..4,
                     plus 0.1 x a standardised 2-D k^-2 random field.
  lognormal_grf_device -- the lognormal_grf recipe drawn with torch on the
                     GPU, for multi-gigabyte fields (the FP64 volume).
"""
import numpy as np

try:
    import scipy.fft as _fft
    _FFT_KW = {"workers": -1}
except Exception:  # pragma: no cover - scipy is present in this image
    _fft = np.fft
    _FFT_KW = {}


def _grf(shape, slope, rng):
    """Standardised periodic Gaussian random field with P(k) ~ k^-slope."""
    shape = tuple(int(s) for s in shape)
    white = rng.standard_normal(shape)
    spec = _fft.rfftn(white, **_FFT_KW)
    del white
    k2 = None
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            f = np.fft.rfftfreq(n) * n
        else:
            f = np.fft.fftfreq(n) * n
        sh = [1] * len(shape)
        sh[ax] = f.size
        term = (f.astype(np.float64) ** 2).reshape(sh)
        k2 = term if k2 is None else k2 + term
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-slope / 4.0), 0.0)  # |k|^(-slope/2)
    spec *= amp
    del amp, k2
    g = _fft.irfftn(spec, s=shape, **_FFT_KW)
    del spec
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def _zero_out(x, frac, rng):
    nz = int(round(frac * x.size))
    if nz > 0:
        idx = rng.choice(x.size, size=nz, replace=False)
        x.reshape(-1)[idx] = 0


def lognormal_grf(shape, seed=0, decades=8.0, neg_frac=0.10, zero_frac=0.005, slope=3.0,
                  dtype=np.float32):
    rng = np.random.default_rng(seed)
    g = _grf(shape, slope, rng)
    gm = np.abs(g).max()
    if gm > 0:
        g *= (decades / 2.0) / gm
    mag = np.power(10.0, g)
    del g
    if neg_frac > 0:
        s = _grf(shape, slope, rng)
        thr = np.quantile(s, 1.0 - neg_frac)
        mag[s > thr] *= -1.0
        del s
    x = mag.astype(dtype)
    del mag
    _zero_out(x, zero_frac, rng)
    return x


def gaussian_bumps(shape, seed=0, zero_frac=0.01, n_bumps=8, n_modes=3, dtype=np.float32):
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    x = np.zeros(shape)
    for _ in range(n_bumps):
        c = [rng.uniform(0, n) for n in shape]
        sig = rng.uniform(4.0, 16.0)
        amp = 10.0 ** rng.uniform(-3.0, 3.0) * (1.0 if rng.random() < 0.5 else -1.0)
        r2 = sum((gq - cq) ** 2 for gq, cq in zip(grids, c))
        x += amp * np.exp(-r2 / (2.0 * sig * sig))
    for _ in range(n_modes):
        k = rng.integers(1, 5, size=len(shape))
        ph = rng.uniform(0.0, 2.0 * np.pi)
        arg = sum(2.0 * np.pi * kq * gq / n for kq, gq, n in zip(k, grids, shape))
        x += np.sin(arg + ph)
    x = x.astype(dtype)
    _zero_out(x, zero_frac, rng)
    return x


def zonal_bands_2d(shape=(1800, 3600), seed=0, noise=0.1, dtype=np.float32):
    rng = np.random.default_rng(seed)
    nlat, nlon = shape
    lat = (np.arange(nlat, dtype=np.float64) + 0.5) / nlat
    band = sum((1.0 / j) * np.cos(2.0 * np.pi * j * lat) for j in range(1, 5))
    x = band[:, None] + noise * _grf(shape, 2.0, rng)
    return x.astype(dtype)


def batch_shapes(n_fields=2000, seed=3000, lo2=128, hi2=1024, lo3=32, hi3=256):
    """Uneven shapes of the batched workload: even index 2-D, odd 3-D, sides
    independent uniform integers."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_fields):
        if i % 2 == 0:
            out.append(tuple(int(v) for v in rng.integers(lo2, hi2 + 1, size=2)))
        else:
            out.append(tuple(int(v) for v in rng.integers(lo3, hi3 + 1, size=3)))
    return out


def lognormal_grf_device(shape, seed=0, decades=8.0, neg_frac=0.10, zero_frac=0.005, slope=3.0,
                         dtype=None, device="cuda", pad_pow2=False):
    """The lognormal_grf recipe drawn on the GPU with torch (for fields of
    gigabytes, where the host FFT would take minutes).  The numbers differ
    from lognormal_grf's (another generator) but follow the same recipe; the
    sign threshold is the (1 - neg_frac) quantile of a 2^24-value subsample of
    its field.  pad_pow2: each Gaussian field is drawn on the grid of the
    next powers of two and cropped to `shape` (one FFT plan per power-of-two
    shape instead of one per shape, for batches of many uneven shapes).
    Returns a torch tensor on `device`."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    shape = tuple(int(s) for s in shape)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))

    gshape = tuple(1 << max(0, (n - 1).bit_length()) for n in shape) if pad_pow2 else shape

    def grf():
        white = torch.randn(gshape, generator=gen, device=device, dtype=torch.float64)
        spec = torch.fft.rfftn(white)
        del white
        k2 = None
        for ax, n in enumerate(gshape):
            if ax == len(gshape) - 1:
                f = torch.fft.rfftfreq(n, device=device, dtype=torch.float64) * n
            else:
                f = torch.fft.fftfreq(n, device=device, dtype=torch.float64) * n
            sh = [1] * len(shape)
            sh[ax] = f.numel()
            term = (f * f).reshape(sh)
            k2 = term if k2 is None else k2 + term
        amp = torch.where(k2 > 0, k2.clamp_min(1e-300) ** (-slope / 4.0),
                          torch.zeros((), dtype=torch.float64, device=device))
        spec *= amp
        del amp, k2
        g = torch.fft.irfftn(spec, s=gshape)
        del spec
        if gshape != shape:
            g = g[tuple(slice(0, n) for n in shape)].contiguous()
        g -= g.mean()
        sd = g.std()
        if sd > 0:
            g /= sd
        return g

    g = grf()
    gm = g.abs().max()
    if gm > 0:
        g *= (decades / 2.0) / gm
    mag = torch.pow(10.0, g)
    del g
    if neg_frac > 0:
        s = grf()
        flat = s.reshape(-1)
        pick = torch.randint(0, flat.numel(), (min(flat.numel(), 1 << 24),), generator=gen,
                             device=device)
        thr = torch.quantile(flat[pick].float(), 1.0 - neg_frac).double()
        mag[s > thr] *= -1.0
        del s, flat, pick
    x = mag.to(dtype)
    del mag
    nz = int(round(zero_frac * x.numel()))
    if nz > 0:
        idx = torch.randperm(x.numel(), generator=gen, device=device)[:nz]
        x.view(-1)[idx] = 0
    return x
