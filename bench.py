#!/usr/bin/env python3
"""Benchmark of the PW_REL perceptron codec on one MI355X.

Workload: a 512^3 FP32 log-normal field (k^-3 Gaussian random field over 8
decades, 10% negative connected regions, 0.5% zeros; seeded synthetic stand-in
for the paper's seismic volumes), block 8^3, point-wise relative bound 1e-2.

Learned path (timed): a network of hidden width 32 is trained on the device
from 1% of the field's points (outside the timed region; its time is
reported), then one step = compress (statistics, constants, grid values and
bound checks of every value, then the fused BF16 matrix-core prediction /
per-block Lorenzo judge / quantisation kernel, scan, raw scatter, header)
followed by decompress (scan, grid values of the raw values, pencil-ordered
reconstruction, inverse map) of the whole field, inputs resident in HBM.  The
plain path (FP32 network H = 16, no judge) is timed the same way for
comparison.  Prints one JSON line.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# vector ALU peak without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (fma)
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12


def compress_flops_per_point(H, K):
    """Algorithmic FP32 + FP64 operations of the fused compression kernel per
    point: log-domain transform (atanh series: 1 div, 10 fma, 5 mul/add; then
    + log2 factor, * 1/w), verification (exp2 Taylor: 4 ops + 13 fma; |x - x^|
    and eps |x|), perceptron (K*H fma, H leaky products, H fma).  fma = 2."""
    transform = 1 + 20 + 5 + 2
    verify = 4 + 26 + 2
    net = 2 * K * H + H + 2 * H  # H = 0: the network runs on the matrix cores
    return transform + verify + net


COMPRESS_SOURCES = ["paper_2309_09778_amd/csrc/pwrel_compress.hip",
                    "paper_2309_09778_amd/csrc/pwrel_kernels.h",
                    "paper_2309_09778_amd/csrc/pwrel_bf16.h",
                    "paper_2309_09778_amd/csrc/pwrel_device.h"]
DECODE_SOURCES = ["paper_2309_09778_amd/csrc/pwrel_decode.hip",
                  "paper_2309_09778_amd/csrc/pwrel_kernels.h",
                  "paper_2309_09778_amd/csrc/pwrel_bf16.h",
                  "paper_2309_09778_amd/csrc/pwrel_device.h"]
COMPRESS_PROFILE = "k_grid_entries_k_compress_learned_bf16_judge_512cubed_f32_eps1e-2.txt"
DECODE_PROFILE = "k_decode_pencil_learned_bf16_judge_512cubed_f32_eps1e-2.txt"


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(summary, files):
    """HBM bytes per launch from a committed rocprofv3 summary (FETCH_SIZE and
    WRITE_SIZE, calibrated on a copy kernel), or None if the kernel's sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        for key in ("traffic_bytes_per_launch:", "source_hash:"):
            if line.startswith(key):
                vals[key] = line.split(":", 1)[1].strip()
    if vals.get("source_hash:") != source_hash(files):
        return None
    return int(vals["traffic_bytes_per_launch:"]) if "traffic_bytes_per_launch:" in vals else None


def huffman_stream_bytes(h, hist, huffman_bits):
    """Compressed size with the codes Huffman-coded: header + model + per-block
    counts + coded bits + codebook (2-byte symbol + 1-byte length per used
    code) + raw values."""
    bits, _ = huffman_bits(hist)
    used = int((hist > 0).sum())
    return (h["off_counts"] + 4 * h["nblocks"] + (bits + 7) // 8 + 3 * used +
            h["n_raw"] * (4 if h["dtype"] == 0 else 8))


def cpu_baseline(x, eps, block, model, side=256):
    """The CPU oracle (single thread) on a sub-cube of the same field: the
    learned mode (both predictors and the per-block judge, the network in
    FP32), compress then decompress."""
    import numpy as np
    from oracle import oracle as O
    sub = np.ascontiguousarray(x[:side, :side, :side])
    m = dict(model, precision=0)
    t0 = time.perf_counter()
    r = O.compress(sub, eps, block, m, O.MODE_LEARNED)
    t1 = time.perf_counter()
    O.decompress(r["codes"], r["raw"], r["consts"], sub.shape, sub.dtype, block, m,
                 O.MODE_LEARNED, flags=r["flags"])
    t2 = time.perf_counter()
    gb = sub.nbytes / 1e9
    return {"value": round(gb / (t2 - t0), 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{side}^3 FP32 sub-cube (first corner) of the same field, learned mode "
                      f"(network H={len(model['b1'])} in FP32 + Lorenzo judge), compress + "
                      f"decompress, single thread",
            "compress_GBps": round(gb / (t1 - t0), 5),
            "decompress_GBps": round(gb / (t2 - t1), 5)}


def run_path(ctx, xd, eps, B, model, judge, ind, out, xh, steps, warmup, pwrel, torch,
             entropy=False):
    """Warm up, then time `steps` round trips (compress + decompress) of one
    path; returns wall times, per-phase device times and the last stream."""
    model = pwrel.model_struct(model)  # the C struct, built once
    for _ in range(warmup):
        s = ctx.compress(xd, eps, B, model, judge=judge, out=out, independent=ind,
                         entropy=entropy)
        ctx.decompress(s, out=xh)
    torch.cuda.synchronize()
    # no garbage-collector pause of this interpreter inside the timed steps
    gc.collect()
    gc.disable()
    ctx.set_profiling(True)
    phase_sum = {k: 0.0 for k in pwrel.PHASES}
    tc = td = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        s = ctx.compress(xd, eps, B, model, judge=judge, out=out, independent=ind,
                         entropy=entropy)
        b = time.perf_counter()
        ctx.decompress(s, out=xh)
        torch.cuda.synchronize()
        c = time.perf_counter()
        tc += b - a
        td += c - b
        for k, v in ctx.phase_times().items():
            phase_sum[k] += v
    t1 = time.perf_counter()
    gc.enable()
    ctx.set_profiling(False)
    return {"wall_s": t1 - t0, "tc": tc, "td": td,
            "phase_ms": {k: v / steps for k, v in phase_sum.items()}, "stream": s}


def stream_stats(ctx, s, x_nbytes, pwrel):
    h = pwrel.header(s)
    sec = pwrel.sections(s)
    hist = ctx.histogram(sec["codes"])
    hbytes = huffman_stream_bytes(h, hist, pwrel.huffman_bits)
    out = {"ratio_stream": round(x_nbytes / h["total_size"], 4),
           "ratio_huffman": round(x_nbytes / hbytes, 4),
           "paper_CR_percent_huffman": round(100.0 * hbytes / x_nbytes, 3),
           "unpredictable_frac": round(h["n_raw"] / h["n"], 7), "n_raw": int(h["n_raw"])}
    if "bflags" in sec:
        out["network_block_frac"] = round(float(sec["bflags"].float().mean()), 4)
    return out


def bound_ok(xd, xh, eps, torch):
    xt, ht = xd.double(), xh.double()
    nz = xt != 0
    return bool(torch.all((xt - ht).abs() <= eps * xt.abs())) and \
        bool(torch.all(ht[~nz] == 0)) and \
        bool(torch.all(torch.signbit(ht[nz]) == torch.signbit(xt[nz])))


def error_stats(ctx, xd, xh, stream, torch, pwrel):
    """Max relative error of x^ (FP64, over non-zero x) and the RMS prediction
    error in grid units (from the code histogram: e = code - 2^15, balance
    points excluded)."""
    import numpy as np
    xt, ht = xd.double(), xh.double()
    nz = xt != 0
    rel = float(((xt[nz] - ht[nz]).abs() / xt[nz].abs()).max())
    hist = ctx.histogram(pwrel.sections(stream)["codes"]).astype(np.float64)
    e = np.arange(65536, dtype=np.float64) - 32768.0
    h = hist.copy()
    h[0] = 0.0
    rms = float(np.sqrt((h * e * e).sum() / max(h.sum(), 1.0)))
    return {"max_rel_error": rel, "pred_error_rms": round(rms, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--side", type=int, default=512)
    ap.add_argument("--block", type=int, default=8)
    ap.add_argument("--hidden", type=int, default=32, help="hidden width of the learned network")
    ap.add_argument("--plain-hidden", type=int, default=16,
                    help="hidden width of the plain FP32 network")
    ap.add_argument("--rho", type=float, default=0.01, help="training sample rate")
    ap.add_argument("--independent", action="store_true",
                    help="blocks predicted without neighbours outside the block (every block "
                         "decodes on its own)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison")
    ap.add_argument("--no-alt", action="store_true",
                    help="skip the learned path with independent blocks (context)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--entropy", action="store_true", help="Huffman-coded streams")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the codec has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_09778_amd import pwrel, synth

    S, eps, B, ind = args.side, args.eps, args.block, args.independent
    x = synth.lognormal_grf((S, S, S), seed=1001)
    print(f"[bench] field {S}^3 FP32 generated", file=sys.stderr, flush=True)
    xd = torch.from_numpy(x).cuda()
    ctx = pwrel.Context(0)
    cap = pwrel.compress_bound(x.shape, pwrel.F32, B)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    xh = torch.empty_like(xd)
    # a plain device copy of known size (HBM counter calibration for profiles)
    xd.clone()
    torch.cuda.synchronize()
    gb = x.nbytes / 1e9
    K = args.steps

    # training (outside the timed region, reported on its own)
    t0 = time.perf_counter()
    learned, rep = ctx.train(xd, eps, B, rho=args.rho, seed=1001, hidden=args.hidden,
                             precision=1, independent=ind)
    train_wall_ms = (time.perf_counter() - t0) * 1e3
    print(f"[bench] trained: chosen {rep['chosen']}, {rep['n_train']} pairs, "
          f"{train_wall_ms:.1f} ms", file=sys.stderr, flush=True)

    # timed: the learned path (BF16 matrix-core network + per-block Lorenzo judge)
    L = run_path(ctx, xd, eps, B, learned, True, ind, out, xh, K, args.warmup, pwrel, torch,
                 entropy=args.entropy)
    ok_l = bound_ok(xd, xh, eps, torch)
    st_l = stream_stats(ctx, L["stream"], x.nbytes, pwrel)
    st_l.update(error_stats(ctx, xd, xh, L["stream"], torch, pwrel))
    ms_step = L["wall_s"] * 1e3 / K
    value = gb / (L["wall_s"] / K)
    print("[bench] learned path timed", file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain:
        pm = pwrel.mlp_init(3, args.plain_hidden, 0.01, 1001)
        P = run_path(ctx, xd, eps, B, pm, False, ind, out, xh, K, args.warmup, pwrel, torch)
        plain = {"network": f"FP32 H={args.plain_hidden}, Lorenzo-initialised (untrained)",
                 "round_trip_GBps": round(gb / (P["wall_s"] / K), 3),
                 "compress_GBps": round(gb / (P["tc"] / K), 3),
                 "decompress_GBps": round(gb / (P["td"] / K), 3),
                 "phase_ms": {k: round(v, 4) for k, v in P["phase_ms"].items()},
                 "bound_ok_every_point": bound_ok(xd, xh, eps, torch)}
        plain.update(stream_stats(ctx, P["stream"], x.nbytes, pwrel))
        plain.update(error_stats(ctx, xd, xh, P["stream"], torch, pwrel))
        print("[bench] plain path timed", file=sys.stderr, flush=True)

    # context: the learned path with independent blocks (each block predicted
    # from its own points only; every block decodes on its own)
    alt = None
    if not args.no_alt and not ind:
        alt_model, alt_rep = ctx.train(xd, eps, B, rho=args.rho, seed=1001, hidden=args.hidden,
                                       precision=1, independent=True)
        A = run_path(ctx, xd, eps, B, alt_model, True, True, out, xh, K, args.warmup, pwrel,
                     torch)
        alt = {"network": f"BF16 H={args.hidden} trained with independent blocks, judge",
               "round_trip_GBps": round(gb / (A["wall_s"] / K), 3),
               "compress_GBps": round(gb / (A["tc"] / K), 3),
               "decompress_GBps": round(gb / (A["td"] / K), 3),
               "phase_ms": {k: round(v, 4) for k, v in A["phase_ms"].items()},
               "bound_ok_every_point": bound_ok(xd, xh, eps, torch)}
        alt.update(stream_stats(ctx, A["stream"], x.nbytes, pwrel))
        alt.update(error_stats(ctx, xd, xh, A["stream"], torch, pwrel))
        print("[bench] learned path with independent blocks timed", file=sys.stderr, flush=True)

    ph = L["phase_ms"]
    N = x.size
    n_raw = st_l["n_raw"]
    nblocks = (S // B) ** 3
    # compression phase (grid values and bound checks, then the fused kernel):
    # ALU-bound (FP64 transform and verification per point; the network runs
    # on the matrix cores)
    flops_pp = compress_flops_per_point(0, 6)
    c_ms = ph["compress"]
    c_ach = flops_pp * N / (c_ms * 1e-3) / 1e12
    c_bytes = N * 4 + N * 2 + nblocks * 5 + n_raw * 4  # field in; codes, counts, flags, raw out
    mfma_useful = 2 * (args.hidden * 6 + args.hidden) * N
    roof_c = {"kernel": "k_grid_entries + k_compress<float,3,8,8,true,1> (a3-a7, BF16 MFMA "
                        "network, judge)", "bound": "alu", "achieved": round(c_ach, 3),
              "peak": round(ALU_PEAK_TFLOPS, 2), "unit": "TFLOP/s",
              "frac": round(c_ach / ALU_PEAK_TFLOPS, 4),
              "traffic": profiled_traffic(COMPRESS_PROFILE, COMPRESS_SOURCES),
              "avg_ms": round(c_ms, 4), "flops_per_point": flops_pp,
              "algorithmic_bytes": c_bytes,
              "hbm_frac": round(c_bytes / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
              "mfma_util": round(mfma_useful / (c_ms * 1e-3) / 2.5e15, 5)}
    # halo-mode decoder (pencils): bound by its chain of dependent pencils;
    # priced against HBM with its algorithmic bytes (codes in, grid values out)
    d_ms = ph["decode_levels"]
    d_bytes = N * 2 + N * 4 + n_raw * 4
    d_ach = d_bytes / (d_ms * 1e-3) / 1e9
    roof_d = {"kernel": "k_decode_pencil<float,8,1> (a8 halo mode, BF16 network, judge)",
              "bound": "hbm", "achieved": round(d_ach, 2), "peak": HBM_PEAK_GBPS,
              "unit": "GB/s", "frac": round(d_ach / HBM_PEAK_GBPS, 5),
              "traffic": profiled_traffic(DECODE_PROFILE, DECODE_SOURCES),
              "avg_ms": round(d_ms, 4), "algorithmic_bytes": d_bytes,
              "limiter": "dependency chain of pencils (levels bz + by)"}
    # the roofline line is the dominant kernel's; the other is reported beside it
    if d_ms >= c_ms:
        roofline, other = roof_d, ("roofline_compress", roof_c)
    else:
        roofline, other = roof_c, ("roofline_decode", roof_d)

    res = {
        "metric": "compress/decompress GB/s at PW_REL 1e-2 and ratio, learned BF16 vs plain FP32",
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+bf16", "data": "synthetic",
        "config": {"workload": f"{S}^3 FP32 log-normal k^-3 GRF (8 decades, 10% negative, "
                               f"0.5% zeros), block {B}^3, eps {eps:g}, learned path: network "
                               f"H={args.hidden} trained on the device ({args.rho:g} sample), "
                               f"BF16 matrix cores, per-block Lorenzo judge" +
                               (", independent blocks" if ind else ", halo prediction"),
                   "path": "learned BF16 (timed) vs plain FP32", "field_bytes": x.nbytes},
        "compress_GBps": round(gb / (L["tc"] / K), 3),
        "decompress_GBps": round(gb / (L["td"] / K), 3),
        "compress_frac_hbm": round(gb / (L["tc"] / K) / HBM_PEAK_GBPS, 4),
        "decompress_frac_hbm": round(gb / (L["td"] / K) / HBM_PEAK_GBPS, 4),
        "phase_ms": {k: round(v, 4) for k, v in ph.items()},
        "bound_ok_every_point": ok_l,
        "training": {"wall_ms": round(train_wall_ms, 2), "ms_sample": round(rep["ms_sample"], 3),
                     "ms_train": round(rep["ms_train"], 3),
                     "ms_select": round(rep["ms_select"], 3), "n_train": rep["n_train"],
                     "n_val": rep["n_val"], "chosen": rep["chosen"],
                     "val_gain_bits": round((rep["val_score"][rep["chosen"]] -
                                             rep["val_score"][0]) / 2.0 ** 32 /
                                            max(rep["n_val"], 1), 4)},
        "roofline": roofline,
        other[0]: other[1],
    }
    res.update(st_l)
    if plain is not None:
        res["plain"] = plain
    if alt is not None:
        res["learned_independent_blocks"] = alt
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(x, eps, B, learned)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
