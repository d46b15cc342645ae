#!/usr/bin/env python3
"""Benchmark of the PW_REL perceptron codec on one MI355X.

Workload: a 512^3 FP32 log-normal field (k^-3 Gaussian random field over 8
decades, 10% negative connected regions, 0.5% zeros; seeded synthetic stand-in
for the paper's seismic volumes), block 8^3, point-wise relative bound 1e-2.

Timed path (the `value`): the learned path with every block decoded on its
own (Sec. 4.4.2's sub-block decompression): a network of hidden width 32 is
trained on the device from 1% of the field's points (outside the timed
region; its time is reported, and the end-to-end rate with it), then one step
= compress (statistics, constants, grid values and bound checks, BF16
matrix-core prediction with the per-block Lorenzo judge, quantisation, scan,
raw values, Huffman stage: histogram, codebook, bit packing) followed by
decompress (Huffman decoding, per-block reconstruction, x^) of the whole
field, inputs resident in HBM.  Beside it, timed the same way: the learned
path with halo prediction, and the plain path (FP32 network of width 16
trained by the same device trainer, no judge).  Then the FP64 volume
(1024 x 1024 x 512, eps 1e-4) and the 2-D 1800 x 3600 field on the learned
path, a measured device copy, and the CPU oracle.  Prints one JSON line.
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
    """Algorithmic FP32 + FP64 operations of the compression kernels per
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
                    "paper_2309_09778_amd/csrc/pwrel_device.h",
                    "paper_2309_09778_amd/csrc/pwrel_wavesort.h"]
COMPRESS_PROFILE = "k_grid_entries_k_compress_learned_bf16_judge_512cubed_f32_eps1e-2.txt"


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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(x, eps, block, model, nproc):
    """The CPU oracle as it stands, learned mode (both predictors and the
    per-block judge, the network in FP32), compress then decompress: one
    thread on a 192^3 corner of the field, and one thread per host core each
    on its own disjoint 96^3 piece (the oracle's C routines run outside the
    interpreter lock)."""
    import concurrent.futures as cf
    import numpy as np
    from oracle import oracle as O
    m = dict(model, precision=0)

    def one(sub):
        r = O.compress(sub, eps, block, m, O.MODE_LEARNED)
        O.decompress(r["codes"], r["raw"], r["consts"], sub.shape, sub.dtype, block, m,
                     O.MODE_LEARNED, flags=r["flags"])

    side1 = 192
    sub = np.ascontiguousarray(x[:side1, :side1, :side1])
    t0 = time.perf_counter()
    r = O.compress(sub, eps, block, m, O.MODE_LEARNED)
    t1 = time.perf_counter()
    O.decompress(r["codes"], r["raw"], r["consts"], sub.shape, sub.dtype, block, m,
                 O.MODE_LEARNED, flags=r["flags"])
    t2 = time.perf_counter()
    gb1 = sub.nbytes / 1e9
    side = 96
    per = x.shape[0] // side
    pieces = []
    for i in range(nproc):
        a, b, c = i % per, (i // per) % per, (i // (per * per)) % per
        pieces.append(np.ascontiguousarray(x[a * side:(a + 1) * side, b * side:(b + 1) * side,
                                             c * side:(c + 1) * side]))
    t3 = time.perf_counter()
    with cf.ThreadPoolExecutor(nproc) as ex:
        list(ex.map(one, pieces))
    t4 = time.perf_counter()
    gbn = sum(p.nbytes for p in pieces) / 1e9
    return {"value": round(gbn / (t4 - t3), 5), "unit": "GB/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nproc} disjoint {side}^3 FP32 pieces of the same field, one host thread "
                      f"each, learned mode (network H={len(model['b1'])} in FP32 + Lorenzo "
                      f"judge), compress + decompress round trip; single thread: {side1}^3 corner",
            "single_thread_GBps": round(gb1 / (t2 - t0), 5),
            "single_thread_compress_GBps": round(gb1 / (t1 - t0), 5),
            "single_thread_decompress_GBps": round(gb1 / (t2 - t1), 5)}


def copy_bandwidth(xd, torch, reps=10):
    """Measured HBM bandwidth of a device copy of the field (bytes read +
    written / time, HIP events)."""
    y = torch.empty_like(xd)
    y.copy_(xd)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(xd)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del y
    return round(2 * xd.numel() * xd.element_size() / (ms * 1e-3) / 1e9, 1)


def run_path(ctx, xd, eps, B, model, judge, ind, entropy, out, xh, steps, warmup, pwrel, torch,
             codebook=None):
    """Warm up, then time `steps` round trips (compress + decompress) of one
    path; returns wall times, per-phase device times and the last stream.
    codebook: a trained Huffman table (else the field's own when entropy)."""
    model = pwrel.model_struct(model) if model is not None else None
    use_net = model is not None
    kw = dict(use_net=use_net, judge=judge, independent=ind, entropy=entropy, out=out,
              codebook=codebook)
    for _ in range(warmup):
        s = ctx.compress(xd, eps, B, model, **kw)
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
        s = ctx.compress(xd, eps, B, model, **kw)
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


def bound_ok(xd, xh, eps, torch):
    """|x - x^| <= eps |x|, sign and zero preserved, on every point (FP64)."""
    ok = True
    n = xd.numel()
    step = 1 << 26
    xf, hf = xd.reshape(-1), xh.reshape(-1)
    for i in range(0, n, step):
        xt, ht = xf[i:i + step].double(), hf[i:i + step].double()
        nz = xt != 0
        ok = ok and bool(torch.all((xt - ht).abs() <= eps * xt.abs())) and \
            bool(torch.all(ht[~nz] == 0)) and \
            bool(torch.all(torch.signbit(ht[nz]) == torch.signbit(xt[nz])))
    return ok


def max_rel_error(xd, xh, torch):
    m = 0.0
    n = xd.numel()
    step = 1 << 26
    xf, hf = xd.reshape(-1), xh.reshape(-1)
    for i in range(0, n, step):
        xt, ht = xf[i:i + step].double(), hf[i:i + step].double()
        nz = xt != 0
        if bool(nz.any()):
            m = max(m, float(((xt[nz] - ht[nz]).abs() / xt[nz].abs()).max()))
    return m


def stream_stats(ctx, s, x_nbytes, pwrel, plain_codes=None):
    """Ratio of the stream as stored (and, for a 16-bit-code stream, the exact
    Huffman estimate), balance points, blocks that keep the network, and the
    RMS prediction error in grid units (from the code histogram)."""
    import numpy as np
    sec = pwrel.sections(s)
    h = sec["header"]
    out = {"ratio_stream": round(x_nbytes / h["total_size"], 4),
           "paper_CR_percent": round(100.0 * h["total_size"] / x_nbytes, 3),
           "stream_bytes": int(h["total_size"]),
           "huffman_coded": bool(h["flags"] & pwrel.HF_HUFFMAN),
           "unpredictable_frac": round(h["n_raw"] / h["n"], 7), "n_raw": int(h["n_raw"])}
    if h["flags"] & pwrel.HF_HUFFMAN:
        out["bits_per_value"] = round(h["n_bits"] / h["n"], 4)
        out["codebook_symbols"] = int(h["n_sym"])
    if "bflags" in sec:
        out["network_block_frac"] = round(float(sec["bflags"].float().mean()), 4)
    return out


def datablocks_leg(ctx, xd, eps, model, steps, warmup, pwrel, torch):
    """The field split into data blocks (sub-volumes) of edge 128 and 64, each
    its own stream with its own factors (Sec. 5), learned BF16 network with
    the judge, independent blocks, 16-bit codes: compress (gather + one
    batched compression) and decompress (per-stream decoding + scatter)
    times, the streams' total size against one stream of the whole field, and
    the bound on every point."""
    gb = xd.numel() * 4 / 1e9
    one = ctx.compress(xd, eps, 8, model, judge=True, independent=True).numel()
    rec = {}
    for sub in (128, 64):
        for _ in range(warmup):
            outs, sizes = ctx.compress_datablocks(xd, eps, sub, model, judge=True,
                                                  independent=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            outs, sizes = ctx.compress_datablocks(xd, eps, sub, model, judge=True,
                                                  independent=True)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - t0) / steps
        hs = sizes.cpu()
        back = ctx.decompress_datablocks(outs, hs, tuple(xd.shape), sub)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            back = ctx.decompress_datablocks(outs, hs, tuple(xd.shape), sub, out=back)
        torch.cuda.synchronize()
        td = (time.perf_counter() - t0) / steps
        total = int(hs.sum().item())
        rec[f"edge_{sub}"] = {"data_blocks": int(outs.shape[0]),
                              "compress_GBps": round(gb / tc, 3),
                              "decompress_GBps": round(gb / td, 3),
                              "ratio_16bit_codes": round(xd.numel() * 4 / total, 4),
                              "size_vs_one_stream": round(total / one, 4),
                              "bound_ok_every_point": bound_ok(xd, back, eps, torch)}
        del outs, back
    return rec


def bf16_vs_fp32(ctx, xd, eps, B, model, out, pwrel, torch):
    """The same trained network on the matrix cores (BF16 operands) and on the
    vector ALU (FP32), no judge: where both code a point, the codes differ by
    the difference of the two rounded predictions (grid units).  Returns the
    largest difference and the share of points where they differ."""
    a = ctx.compress(xd, eps, B, dict(model, precision=1), independent=True, out=out)
    ca = pwrel.sections(a)["codes"].clone()
    b = ctx.compress(xd, eps, B, dict(model, precision=0), independent=True, out=out)
    cb = pwrel.sections(b)["codes"]
    ia = ca.view(torch.int16).to(torch.int32) & 0xFFFF
    ib = cb.view(torch.int16).to(torch.int32) & 0xFFFF
    both = (ia != 0) & (ib != 0)
    d = (ia - ib).abs()[both]
    return {"max_code_diff": int(d.max().item()) if d.numel() else 0,
            "frac_points_differ": round(float((d != 0).float().mean().item()), 6),
            "points_compared": int(d.numel())}


def pred_error_rms(ctx, codes_t, pwrel):
    import numpy as np
    hist = ctx.histogram(codes_t).astype(np.float64)
    e = np.arange(65536, dtype=np.float64) - 32768.0
    hist[0] = 0.0
    return round(float(np.sqrt((hist * e * e).sum() / max(hist.sum(), 1.0))), 4)


def path_record(name, P, ctx, xd, xh, eps, gb, K, pwrel, torch):
    rec = {"path": name,
           "round_trip_GBps": round(gb / (P["wall_s"] / K), 3),
           "compress_GBps": round(gb / (P["tc"] / K), 3),
           "decompress_GBps": round(gb / (P["td"] / K), 3),
           "ms_per_step": round(P["wall_s"] * 1e3 / K, 4),
           "phase_ms": {k: round(v, 4) for k, v in P["phase_ms"].items()},
           "bound_ok_every_point": bound_ok(xd, xh, eps, torch),
           "max_rel_error": max_rel_error(xd, xh, torch)}
    rec.update(stream_stats(ctx, P["stream"], xd.numel() * xd.element_size(), pwrel))
    return rec


def train_record(rep, wall_ms):
    return {"wall_ms": round(wall_ms, 2), "ms_sample": round(rep["ms_sample"], 3),
            "ms_train": round(rep["ms_train"], 3), "ms_select": round(rep["ms_select"], 3),
            "n_train": rep["n_train"], "n_val": rep["n_val"], "chosen": rep["chosen"],
            "train_pairs_per_s": round(rep["n_train"] / max(rep["ms_train"], 1e-9) * 1e3, 1),
            "val_gain_bits": round((rep["val_score"][rep["chosen"]] - rep["val_score"][0]) /
                                   2.0 ** 32 / max(rep["n_val"], 1), 4)}


def batch_leg(ctx, n_fields, eps, steps, warmup, hidden, plain_hidden, rho, pwrel, synth, torch):
    """Many uneven fields in one batched call: n_fields FP32 fields, even
    index 2-D (sides uniform in 128..1024), odd 3-D (sides uniform in
    32..256), each a log-normal k^-3 field of its own seed with 5% negative
    regions; eps, independent blocks.  Two paths: the learned one (BF16
    network of width `hidden` and the per-block judge) and the plain one
    (FP32 network of width `plain_hidden`, no judge), each network trained on
    the device on the first field of its dimensionality.  Per path: the
    tile autotuner, eager calls, graph replays, and the same fields
    compressed one call each (the unbatched baseline); a sample of fields
    is checked byte for byte against single-field compression and decoded
    against the bound."""
    import numpy as np
    shapes = synth.batch_shapes(n_fields, seed=3000)
    t0 = time.perf_counter()
    xs = []
    for i, s in enumerate(shapes):
        xs.append(synth.lognormal_grf_device(s, seed=3000 + i, decades=8.0, neg_frac=0.05,
                                             zero_frac=0.005, pad_pow2=True))
        if (i + 1) % 100 == 0:
            log(f"batch fields generated: {i + 1}/{n_fields}")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nvals = sum(x.numel() for x in xs)
    gb = nvals * 4 / 1e9
    i3 = next(i for i, s in enumerate(shapes) if len(s) == 3)
    i2 = next(i for i, s in enumerate(shapes) if len(s) == 2)
    outs = [torch.empty(pwrel.compress_bound(x.shape, pwrel.F32, 8 if x.dim() == 3 else 16),
                        dtype=torch.uint8, device="cuda") for x in xs]
    sizes = torch.zeros(len(xs), dtype=torch.int64, device="cuda")
    rec = {"fields": n_fields, "values": nvals, "bytes": nvals * 4,
           "fields_3d": sum(len(s) == 3 for s in shapes), "generate_s": round(gen_s, 2),
           "workload": f"{n_fields} FP32 fields: even index 2-D (sides uniform 128..1024, block "
                       f"16^2), odd 3-D (sides uniform 32..256, block 8^3); log-normal k^-3 "
                       f"field per seed (drawn on the next power-of-two grid and cropped), 8 decades, 5% "
                       f"negative regions, 0.5% zeros; eps "
                       f"{eps:g}; independent blocks; 16-bit codes"}
    sample = sorted(set([0, 1, 2, 3] + list(range(0, n_fields, max(1, n_fields // 16)))))
    for name, H, prec, judge in (("learned", hidden, 1, True), ("plain", plain_hidden, 0, False)):
        models, train_ms = {}, 0.0
        for nd, i in ((3, i3), (2, i2)):
            a = time.perf_counter()
            m, _ = ctx.train(xs[i], eps, 8 if nd == 3 else 16, rho=rho, seed=3000 + i, hidden=H,
                             precision=prec, independent=True)
            train_ms += (time.perf_counter() - a) * 1e3
            models[nd] = m
        req = ctx.batch_request(xs, eps, models=models, judge=judge, independent=True, outs=outs,
                                sizes=sizes)
        variants, tune_ms = req.tune(reps=3)
        for _ in range(warmup):
            req.run()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(steps):
            req.run()
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - a) * 1e3 / steps
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                req.run(stream=side)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - a) * 1e3 / steps
        views = req.views()
        sz = [int(v.numel()) for v in views]
        # the same fields one call each (each call synchronises once)
        mst = {nd: pwrel.model_struct(m) for nd, m in models.items()}
        a = time.perf_counter()
        for x, o in zip(xs, outs):
            ctx.compress(x, eps, 8 if x.dim() == 3 else 16, mst[x.dim()], judge=judge,
                         independent=True, out=o)
        torch.cuda.synchronize()
        single_ms = (time.perf_counter() - a) * 1e3
        # the batch again, then the sample: byte-identical to single calls, and decoded
        req.run()
        views = req.views()
        same, bound = True, True
        for i in sample:
            x = xs[i]
            s1 = ctx.compress(x, eps, 8 if x.dim() == 3 else 16, models[x.dim()], judge=judge,
                              independent=True)
            same = same and s1.numel() == views[i].numel() and bool(torch.equal(s1, views[i]))
            xh = ctx.decompress(views[i])
            bound = bound and bound_ok(x, xh, eps, torch)
        shp = ctx.batch_tiles()[1]
        rec[name] = {
            "path": ("BF16 H=%d network + per-block judge" if judge else
                     "FP32 H=%d network, no judge") % H,
            "eager_ms": round(eager_ms, 3), "graph_ms": round(graph_ms, 3),
            "eager_GBps": round(gb / (eager_ms * 1e-3), 2),
            "graph_GBps": round(gb / (graph_ms * 1e-3), 2),
            "unbatched_ms": round(single_ms, 2),
            "speedup_vs_unbatched": round(single_ms / graph_ms, 2),
            "ratio_16bit_codes": round(nvals * 4 / max(sum(sz), 1), 4),
            "failed_fields": int(sum(1 for v in sz if v == 0)),
            "tiles": {"variants_3d_2d": variants, "tile_3d": shp[0], "tile_2d": shp[1],
                      "compress_ms_3d": [round(v, 3) for v in tune_ms[0]],
                      "compress_ms_2d": [round(v, 3) for v in tune_ms[1]]},
            "sample_fields": len(sample), "sample_equal_single": same,
            "sample_bound_ok": bound, "train_ms": round(train_ms, 1)}
        log(f"batch {name}: graph {graph_ms:.2f} ms, eager {eager_ms:.2f} ms, "
            f"unbatched {single_ms:.1f} ms")
        del g
    del xs, outs
    torch.cuda.empty_cache()
    return rec


def openloop_leg(ctx, side, eps, rho, plain_hidden, pwrel, synth, torch):
    """The paper's literal open-loop prediction (raw neighbours, drifting
    decoder) on a side^3 FP32 log-normal field, independent 8^3 blocks:
    Lorenzo and a device-trained FP32 network; m by coverage and m = 16;
    deliberate balance points every gap points (0 = none).  Reports points
    breaking the bound, the largest relative error (in units of eps: the
    paper accepts up to 1.5) and the balance-point share; the grid-snapped
    codec on the same field breaks no bound."""
    x = synth.lognormal_grf_device((side, side, side), seed=1005)
    net, _ = ctx.train(x, eps, 8, rho=rho, seed=1005, hidden=plain_hidden, precision=0,
                       independent=True)
    out = {"field": f"{side}^3 FP32 log-normal k^-3 (8 decades, 10% negative, 0.5% zeros), "
                    f"block 8^3 independent, eps {eps:g}", "runs": []}
    N = x.numel()
    for pred, m in (("lorenzo", None), ("fp32_net_H%d" % plain_hidden, net)):
        for mbits, gap in ((0, 0), (16, 0), (0, 16), (16, 16), (0, 4)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.openloop(x, eps, 8, m, mbits, gap)
            ms = (time.perf_counter() - t0) * 1e3
            rep = r["report"]
            out["runs"].append({
                "predictor": pred, "mbits": rep["mbits"], "m_by_coverage": mbits == 0,
                "gap": gap, "violation_frac": round(rep["violations"] / N, 6),
                "max_rel_over_eps": round(rep["max_rel_error"] / eps, 3),
                "accepted_1p5": rep["max_rel_error"] <= 1.5 * eps,
                "balance_frac": round(rep["n_raw"] / N, 5),
                "coverage_16": round(sum(rep["hist"][:17]) / N, 5), "ms": round(ms, 2)})
            del r
    s = ctx.compress(x, eps, 8, None, use_net=False, independent=True)
    xh = ctx.decompress(s)
    out["grid_snapped_bound_ok"] = bound_ok(x, xh, eps, torch)
    del x, xh, s
    torch.cuda.empty_cache()
    return out


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
    ap.add_argument("--only-timed", action="store_true",
                    help="the timed path only (no other paths, legs or CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-fields", type=int, default=2000,
                    help="fields of the batched leg (0: no batched leg)")
    ap.add_argument("--only-batch", action="store_true",
                    help="the batched leg only (one JSON line with its record)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the codec has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_09778_amd import pwrel, synth

    if args.only_batch:
        ctx = pwrel.Context(0)
        rec = batch_leg(ctx, args.batch_fields, args.eps, args.steps, args.warmup, args.hidden,
                        args.plain_hidden, args.rho, pwrel, synth, torch)
        print(json.dumps({"batch": rec}), flush=True)
        return

    S, eps, B = args.side, args.eps, args.block
    x = synth.lognormal_grf((S, S, S), seed=1001)
    log(f"field {S}^3 FP32 generated")
    xd = torch.from_numpy(x).cuda()
    ctx = pwrel.Context(0)
    cap = pwrel.compress_bound(x.shape, pwrel.F32, B)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    xh = torch.empty_like(xd)
    copy_gbps = copy_bandwidth(xd, torch)
    gb = x.nbytes / 1e9
    K = args.steps
    N = x.size

    # training (outside the timed region, reported on its own)
    t0 = time.perf_counter()
    learned, rep = ctx.train(xd, eps, B, rho=args.rho, seed=1001, hidden=args.hidden,
                             precision=1, independent=True)
    # the Huffman table of the training phase: the compression simulated on
    # a 2 % share of the blocks (the paper's validation share)
    table = ctx.train_codebook(xd, eps, B, learned, judge=True, independent=True, frac=0.02,
                               seed=1001)
    train_ms = (time.perf_counter() - t0) * 1e3
    log(f"trained: chosen {rep['chosen']}, {rep['n_train']} pairs, {train_ms:.1f} ms")

    # timed: the learned path, independent blocks, judge, the codes Huffman
    # coded with the table of the training phase
    L = run_path(ctx, xd, eps, B, learned, True, True, True, out, xh, K, args.warmup, pwrel,
                 torch, codebook=table)
    rec_l = path_record("learned BF16 H=%d, judge, independent blocks, Huffman table of the "
                        "training phase (%d symbols, %d-bit escape)"
                        % (args.hidden, table.n_sym, table.esc_len), L, ctx, xd, xh, eps, gb, K,
                        pwrel, torch)
    ms_step = L["wall_s"] * 1e3 / K
    value = gb / (L["wall_s"] / K)
    # the same call's codes as 16 bits (for the prediction error and the ratio estimate)
    s16 = ctx.compress(xd, eps, B, learned, judge=True, independent=True, out=out)
    rec_l["pred_error_rms"] = pred_error_rms(ctx, pwrel.sections(s16)["codes"], pwrel)
    hist = ctx.histogram(pwrel.sections(s16)["codes"])
    rec_l["huffman_bits_estimate"] = pwrel.huffman_bits(hist)[0]
    rec_l["bf16_vs_fp32_network"] = bf16_vs_fp32(ctx, xd, eps, B, learned, out, pwrel, torch)
    log("learned path timed")

    ph = L["phase_ms"]
    n_raw = rec_l["n_raw"]
    nblocks = (S // B) ** 3
    # compression kernels (grid values and bound checks, then the fused
    # prediction / judge / quantisation kernel): issue-bound on the ALUs
    flops_pp = compress_flops_per_point(0, 6)
    c_ms = ph["compress"]
    c_ach = flops_pp * N / (c_ms * 1e-3) / 1e12
    c_bytes = N * 4 + N * 2 + nblocks * 5 + n_raw * 4  # field in; codes, counts, flags, raw out
    mfma_useful = 2 * (args.hidden * 6 + args.hidden) * N
    roofline = {"kernel": "k_grid_entries + k_compress<float,3,8,8,true,1,false,0,W32> pair (a3-a7, "
                          "BF16 MFMA network, exact per-block judge)", "bound": "alu",
                "achieved": round(c_ach, 3), "peak": round(ALU_PEAK_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(c_ach / ALU_PEAK_TFLOPS, 4),
                "traffic": profiled_traffic(COMPRESS_PROFILE, COMPRESS_SOURCES),
                "avg_ms": round(c_ms, 4), "flops_per_point": flops_pp,
                "algorithmic_bytes": c_bytes,
                "hbm_frac": round(c_bytes / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "mfma_util": round(mfma_useful / (c_ms * 1e-3) / 2.5e15, 5)}
    # the lane decoder (independent blocks): codes in, x^ out
    d_ms = ph["decode_levels"]
    d_bytes = N * 2 + N * 4 + n_raw * 4
    roof_d = {"kernel": "k_decode_lanes<float,3,8,8,1> (a8, one lane per block, BF16 network)",
              "bound": "hbm", "achieved": round(d_bytes / (d_ms * 1e-3) / 1e9, 2),
              "peak": HBM_PEAK_GBPS, "unit": "GB/s",
              "frac": round(d_bytes / (d_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 5),
              "avg_ms": round(d_ms, 4), "algorithmic_bytes": d_bytes}

    res = {
        "metric": "compress/decompress GB/s at PW_REL 1e-2 and ratio, learned BF16 vs plain FP32",
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+bf16", "data": "synthetic",
        "config": {"workload": f"{S}^3 FP32 log-normal k^-3 GRF (8 decades, 10% negative, "
                               f"0.5% zeros), block {B}^3, eps {eps:g}, learned path: network "
                               f"H={args.hidden} trained on the device ({args.rho:g} sample), "
                               f"BF16 matrix cores, per-block Lorenzo judge, independent blocks, "
                               f"Huffman table of the training phase (2 % of the blocks)",
                   "field_bytes": x.nbytes},
        "compress_GBps": rec_l["compress_GBps"], "decompress_GBps": rec_l["decompress_GBps"],
        "compress_frac_hbm": round(rec_l["compress_GBps"] / HBM_PEAK_GBPS, 4),
        "decompress_frac_hbm": round(rec_l["decompress_GBps"] / HBM_PEAK_GBPS, 4),
        "phase_ms": rec_l["phase_ms"], "bound_ok_every_point": rec_l["bound_ok_every_point"],
        "max_rel_error": rec_l["max_rel_error"],
        "ratio_stream": rec_l["ratio_stream"], "paper_CR_percent": rec_l["paper_CR_percent"],
        "bits_per_value": rec_l.get("bits_per_value"), "n_raw": n_raw,
        "network_block_frac": rec_l.get("network_block_frac"),
        "pred_error_rms": rec_l["pred_error_rms"],
        "training": train_record(rep, train_ms),
        "end_to_end_with_training_GBps": round(gb / ((train_ms + ms_step) * 1e-3), 3),
        "roofline": roofline,
        "roofline_decode": roof_d,
        "copy_GBps_measured": copy_gbps,
        "learned": rec_l,
    }
    # the same path with a table built in the call from the field's own
    # code histogram (optimal for the field; a histogram pass and a host
    # build inside every call)
    T = run_path(ctx, xd, eps, B, learned, True, True, True, out, xh, K, args.warmup, pwrel,
                 torch)
    res["learned_own_table"] = path_record(
        "learned BF16 H=%d, judge, independent blocks, Huffman table of the field's own "
        "histogram" % args.hidden, T, ctx, xd, xh, eps, gb, K, pwrel, torch)
    log("learned path with the field's own table timed")
    if args.only_timed:
        print(json.dumps(res), flush=True)
        return

    res["data_blocks"] = datablocks_leg(ctx, xd, eps, learned, K, args.warmup, pwrel, torch)
    log("data-block leg timed")

    # the learned path with halo prediction
    lh, rep_h = ctx.train(xd, eps, B, rho=args.rho, seed=1001, hidden=args.hidden, precision=1)
    th = ctx.train_codebook(xd, eps, B, lh, judge=True, frac=0.02, seed=1001)
    H_ = run_path(ctx, xd, eps, B, lh, True, False, True, out, xh, K, args.warmup, pwrel, torch,
                  codebook=th)
    res["learned_halo"] = path_record("learned BF16 H=%d, judge, halo prediction, Huffman table "
                                      "of the training phase" % args.hidden, H_, ctx, xd, xh, eps,
                                      gb, K, pwrel, torch)
    log("learned halo path timed")

    # the plain path: FP32 network of width 16 trained by the same device trainer
    pm, rep_p = ctx.train(xd, eps, B, rho=args.rho, seed=1001, hidden=args.plain_hidden,
                          precision=0, independent=True)
    tp = ctx.train_codebook(xd, eps, B, pm, independent=True, frac=0.02, seed=1001)
    P = run_path(ctx, xd, eps, B, pm, False, True, True, out, xh, K, args.warmup, pwrel, torch,
                 codebook=tp)
    res["plain"] = path_record("plain FP32 H=%d (trained on the device, no judge), independent "
                               "blocks, Huffman table of the training phase" % args.plain_hidden,
                               P, ctx, xd, xh, eps, gb, K, pwrel, torch)
    res["plain"]["training"] = train_record(rep_p, rep_p["ms_sample"] + rep_p["ms_train"])
    s16 = ctx.compress(xd, eps, B, pm, independent=True, out=out)
    res["plain"]["pred_error_rms"] = pred_error_rms(ctx, pwrel.sections(s16)["codes"], pwrel)
    m0 = pwrel.mlp_init(3, args.plain_hidden, 0.01, 1001)
    t0h = ctx.train_codebook(xd, eps, B, m0, frac=0.02, seed=1001)
    Ph = run_path(ctx, xd, eps, B, m0, False, False, True, out, xh, K, args.warmup, pwrel, torch,
                  codebook=t0h)
    res["lorenzo_halo"] = path_record("untrained network (= one-layer Lorenzo), halo "
                                      "prediction, Huffman table of the training phase", Ph, ctx,
                                      xd, xh, eps, gb, K, pwrel, torch)
    log("plain paths timed")
    res["learned_vs_plain_size"] = round(rec_l["stream_bytes"] / res["plain"]["stream_bytes"], 4)
    cpu_model = learned
    del out, xh
    torch.cuda.empty_cache()

    # the FP64 volume (1024 x 1024 x 512, eps 1e-4) on the learned path
    shp = (512, 1024, 1024)
    x64 = synth.lognormal_grf_device(shp, seed=1004, decades=12, neg_frac=0.10, zero_frac=0.01,
                                     dtype=torch.float64)
    o64 = torch.empty(pwrel.compress_bound(shp, pwrel.F64, 8), dtype=torch.uint8, device="cuda")
    h64 = torch.empty_like(x64)
    t0 = time.perf_counter()
    m64, rep64 = ctx.train(x64, 1e-4, 8, rho=0.002, seed=1004, hidden=args.hidden, precision=1,
                           independent=True)
    t64tab = ctx.train_codebook(x64, 1e-4, 8, m64, judge=True, independent=True, frac=0.02,
                                seed=1004)
    t64 = (time.perf_counter() - t0) * 1e3
    F = run_path(ctx, x64, 1e-4, 8, m64, True, True, True, o64, h64, 3, 1, pwrel, torch,
                 codebook=t64tab)
    res["fp64_volume"] = path_record("FP64 1024x1024x512 (12 decades, 10% negative, 1% zeros), "
                                     "eps 1e-4, learned BF16, judge, independent blocks, Huffman "
                                     "table of the training phase",
                                     F, ctx, x64, h64, 1e-4, x64.numel() * 8 / 1e9, 3, pwrel,
                                     torch)
    res["fp64_volume"]["training"] = train_record(rep64, t64)
    log("FP64 volume timed")
    del x64, o64, h64, F
    torch.cuda.empty_cache()

    # the 2-D 1800 x 3600 field (zonal bands + k^-2 noise), block 16^2, learned path
    x2 = torch.from_numpy(synth.zonal_bands_2d((1800, 3600), seed=1002)).cuda()
    o2 = torch.empty(pwrel.compress_bound(x2.shape, pwrel.F32, 16), dtype=torch.uint8,
                     device="cuda")
    h2 = torch.empty_like(x2)
    m2, rep2 = ctx.train(x2, eps, 16, rho=args.rho, seed=1002, hidden=args.hidden, precision=1,
                         independent=True)
    t2 = ctx.train_codebook(x2, eps, 16, m2, judge=True, independent=True, frac=0.02, seed=1002)
    Z = run_path(ctx, x2, eps, 16, m2, True, True, True, o2, h2, K, args.warmup, pwrel, torch,
                 codebook=t2)
    res["zonal_2d"] = path_record("2-D 1800x3600 zonal bands + k^-2 noise, block 16^2, learned "
                                  "BF16, judge, independent blocks, Huffman table of the training "
                                  "phase", Z, ctx, x2, h2, eps, x2.numel() * 4 / 1e9, K, pwrel,
                                  torch)
    m20 = pwrel.mlp_init(2, args.plain_hidden, 0.01, 1002)
    t20 = ctx.train_codebook(x2, eps, 16, m20, independent=True, frac=0.02, seed=1002)
    Z0 = run_path(ctx, x2, eps, 16, m20, False, True, True, o2, h2, K, args.warmup, pwrel, torch,
                  codebook=t20)
    res["zonal_2d"]["lorenzo_ratio_stream"] = stream_stats(ctx, Z0["stream"], x2.numel() * 4,
                                                           pwrel)["ratio_stream"]
    log("2-D field timed")

    del x2, o2, h2, Z, Z0
    torch.cuda.empty_cache()
    res["open_loop"] = openloop_leg(ctx, 256, eps, args.rho, args.plain_hidden, pwrel, synth,
                                    torch)
    log("open-loop leg measured")
    if args.batch_fields > 0:
        res["batch"] = batch_leg(ctx, args.batch_fields, eps, K, args.warmup, args.hidden,
                                 args.plain_hidden, args.rho, pwrel, synth, torch)
        log("batched leg timed")

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        nproc = min(len(os.sched_getaffinity(0)), 16)
        res["cpu_baseline"] = cpu_baseline(x, eps, B, cpu_model, nproc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
