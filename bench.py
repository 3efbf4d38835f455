#!/usr/bin/env python3
"""Throughput of the w-stacking imager on one MI355X: visibilities imaged per second.

A step is one whole dirty image (all stages: bucket sort, gridding + row FFT, column
FFT + w-phase + stacking + taper) of one synthetic visibility set already resident in HBM.
The default workload is the MeerKAT-shaped single channel: 7 257 600 visibilities,
4096^2 image, 32 w-planes, Kaiser-Bessel support 7, float32 path; the float64 path is
timed on the same inputs and its rate and the float32/float64 speedup are reported too.

With --workload c4 a step is one call that images all 64 channels of the batched
MeerKAT-shaped set (856-1712 MHz, 1024^2 images, 16 w-planes, 0-60 % random flagging per
channel); the same channels imaged by 64 single-channel calls are timed beside it.

With --workload c5 a step is one evaluation of a weighted chi-square data-fidelity loss and
its gradient with respect to a 2048^2 sky image through the differentiable imaging operator
(prediction of 4 M visibilities, then the transpose for the gradient), float32.

Prints ONE JSON line.  Extra objects:
  roofline     : the dominant kernel's algorithmic bytes (or flops) per launch over its
                 average duration, from HIP events recorded on the plan's stream during
                 the timed steps, against the MI355X peak;
  cpu_baseline : the FP64 oracle timed on a bounded sample of the same workload on the
                 host cores (test infrastructure, run only here, rank 0, N = 1).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "visibilities imaged/s (FP32 vs FP64 path, 1 GPU) at ≤1e-5 rel err vs FP64 oracle"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector, published (includes packed issue)
WORKLOADS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_19714_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_traffic(prec: str, n: int, m_kept: int, n_occ: int, strip_rows: int):
    """Bytes each stage must move (not sort scratch re-reads), per call."""
    cb = 8 if prec == "f32" else 16          # complex element
    rb = cb // 2
    rec = 4 + cb + cb                        # record: cell id, sub-cell offsets, W*V
    inter = n_occ * strip_rows * n * cb      # row-transformed occupied strips
    return {
        "grid_rows": m_kept * rec + inter,                   # records in, strips out
        "cols_stack": inter + n * n * rb,                    # strips in, image out
    }


def cols_stack_flops(n: int, nw_occ: int) -> float:
    """Algorithmic flops of the stacking pass: a length-n column FFT per image column and
    plane (5 n log2 n) and a complex multiply by the w-phase plus the accumulate (8)."""
    return nw_occ * n * (5.0 * n * math.log2(n) + 8.0 * n)


# accuracy variants applied to every plan (--fold, --pad2); empty: the plain method
VARIANT = {}


def run_gpu(ds, prec: str, steps: int, warmup: int):
    import torch
    import paper_2601_19714_amd as ws

    d = ds.as_precision(prec)
    dev = torch.device("cuda:0")
    uvw = torch.from_numpy(d.uvw_m).to(dev)
    vis = torch.from_numpy(d.vis).to(dev)
    wts = torch.from_numpy(d.weights).to(dev)
    plan = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, prec, max_vis=d.m, **VARIANT)
    out = torch.empty((d.n, d.n), dtype=torch.float32 if prec == "f32" else torch.float64, device=dev)
    _, st = plan.image(uvw, vis, wts, d.freq_hz, out=out, stats=True)
    for _ in range(warmup):
        plan.image(uvw, vis, wts, d.freq_hz, out=out)
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.image(uvw, vis, wts, d.freq_hz, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = plan.read_timing()
    plan.set_timing(False)
    info = plan.info()
    img = out.cpu().numpy()
    plan.close()
    return {"ms_per_step": 1e3 * wall / steps, "timing": timing, "stats": st, "info": info, "image": img}


def run_gpu_batch(chans, steps: int, warmup: int):
    """All channels in one wsimg_image_batch call per step; then the same channels as one
    wsimg_image call each (the unbatched way), for comparison."""
    import numpy as np
    import torch
    import synth
    import paper_2601_19714_amd as ws

    uvw_h, vis_h, wts_h, counts, freqs = synth.stack_channels(chans)
    dev = torch.device("cuda:0")
    uvw = torch.from_numpy(uvw_h).to(dev)
    vis = torch.from_numpy(vis_h).to(dev)
    wts = torch.from_numpy(wts_h).to(dev)
    d = chans[0]
    nch = len(chans)
    plan = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, "f32", max_vis=sum(counts),
                   max_channels=nch, **VARIANT)
    out = torch.empty((nch, d.n, d.n), dtype=torch.float32, device=dev)
    _, st = plan.image_batch(uvw, vis, wts, counts, freqs, out=out, stats=True)
    for _ in range(warmup):
        plan.image_batch(uvw, vis, wts, counts, freqs, out=out)
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.image_batch(uvw, vis, wts, counts, freqs, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = plan.read_timing()
    plan.set_timing(False)
    info = plan.info()
    plan.close()

    # the same call captured into a HIP graph and replayed
    gplan = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, "f32", max_vis=sum(counts),
                    max_channels=nch, **VARIANT)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gplan.image_batch(uvw, vis, wts, counts, freqs, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gplan.image_batch(uvw, vis, wts, counts, freqs, out=out)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    del graph
    gplan.close()

    off = np.concatenate([[0], np.cumsum(counts)])
    single = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, "f32", max_vis=max(counts), **VARIANT)
    one = torch.empty((d.n, d.n), dtype=torch.float32, device=dev)
    sl = [slice(int(off[c]), int(off[c + 1])) for c in range(nch)]

    def all_single():
        for c in range(nch):
            single.image(uvw[sl[c]], vis[sl[c]], wts[sl[c]], freqs[c], out=one)

    all_single()
    torch.cuda.synchronize()
    s_steps = max(1, steps // 4)
    t0 = time.perf_counter()
    for _ in range(s_steps):
        all_single()
    torch.cuda.synchronize()
    wall_single = time.perf_counter() - t0
    single.close()
    return {"ms_per_step": 1e3 * wall / steps, "timing": timing, "stats": st, "info": info,
            "counts": counts, "ms_per_step_single_calls": 1e3 * wall_single / s_steps,
            "ms_per_step_graph": 1e3 * wall_graph / steps}


def cpu_baseline(ds, n_sample_planes: int):
    """The oracle on a stratified sample of w-planes, scaled to the whole workload:
    vis/s = M / (T_prepare + (Nw / n_sample) * T_sampled_planes)."""
    import numpy as np
    import oracle
    d = ds.as_precision("f64")
    prm = oracle.Params(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta)
    t0 = time.perf_counter()
    pr = oracle.prepare(d.uvw_m, d.weights, d.freq_hz, prm)
    t_prep = time.perf_counter() - t0
    step = max(1, d.n_wplanes // n_sample_planes)
    planes = list(range(0, d.n_wplanes, step))[:n_sample_planes]
    t0 = time.perf_counter()
    oracle.wstack_image(d.uvw_m, d.vis, d.weights, d.freq_hz, prm, planes=planes, prepared=pr)
    t_planes = time.perf_counter() - t0
    est = t_prep + (d.n_wplanes / len(planes)) * t_planes
    m_sample = int(np.isin(pr.k[pr.keep], planes).sum())
    return {
        "value": d.m / est, "unit": "visibilities/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 oracle (steps 1-3 on all {d.m} rows: {t_prep:.2f} s; steps 4-8 on w-planes "
                   f"{planes} of {d.n_wplanes}, {m_sample} rows: {t_planes:.2f} s), whole-image time "
                   f"estimated as prepare + {d.n_wplanes}/{len(planes)} x sampled planes = {est:.1f} s; "
                   f"single-threaded numpy FFT and C gridding loop"),
    }


def read_pmc_traffic(kernel: str, workload: str, src_hash: str):
    """HBM bytes per dispatch from a committed rocprofv3 PMC summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != src_hash:
        return None
    return rec.get("hbm_bytes_per_dispatch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2")
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 path")
    ap.add_argument("--fold", action="store_true", help="w-folding (accuracy variant)")
    ap.add_argument("--pad2", action="store_true", help="grid of twice the image side (accuracy variant)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-planes", type=int, default=4)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (PMC byte-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this imager runs on a single device (multi-GPU sharding "
              "is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "copies": 5}))
        return

    if args.fold:
        VARIANT["fold_w"] = True
    if args.pad2:
        VARIANT["pad"] = 2
    cfg = WORKLOADS[args.workload]
    if cfg == 4:
        bench_batch(args)
        return
    if cfg == 5:
        bench_adjoint(args)
        return
    t0 = time.perf_counter()
    ds = synth.make_config(cfg, device="cuda" if torch.cuda.is_available() else "cpu")
    log(f"generated {ds.name}: M={ds.m} n={ds.n} nw={ds.n_wplanes} W={ds.support} "
        f"in {time.perf_counter() - t0:.1f}s")

    r32 = run_gpu(ds, "f32", args.steps, args.warmup)
    log(f"f32: {r32['ms_per_step']:.3f} ms/step  stages(ms/call) " +
        ", ".join(f"{k}={v / max(1, r32['timing']['calls']):.4f}" for k, v in r32["timing"]["ms"].items()))
    r64 = None
    if not args.no_f64:
        r64 = run_gpu(ds, "f64", args.steps, args.warmup)
        log(f"f64: {r64['ms_per_step']:.3f} ms/step  stages(ms/call) " +
            ", ".join(f"{k}={v / max(1, r64['timing']['calls']):.4f}" for k, v in r64["timing"]["ms"].items()))

    m = ds.m
    value = m / (r32["ms_per_step"] / 1e3)
    st = r32["stats"]
    calls = max(1, r32["timing"]["calls"])
    per_call = {k: v / calls for k, v in r32["timing"]["ms"].items()}
    dominant = max(per_call, key=per_call.get)
    nw_occ = st["n_planes_occupied"]
    traffic = algorithmic_traffic("f32", ds.n, st["n_gridded"], st["n_strips_occupied"], r32["info"]["strip_rows"])
    src_hash = kernel_source_hash()
    roof = None
    if dominant in traffic:
        achieved_gbs = traffic[dominant] / (per_call[dominant] / 1e3) / 1e9
        roof_hbm = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved_gbs / HBM_PEAK_GBS}
        roof = roof_hbm
        if dominant == "cols_stack":
            tf = cols_stack_flops(ds.n, nw_occ) / (per_call[dominant] / 1e3) / 1e12
            roof_alu = {"bound": "alu", "achieved": tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / FP32_VECTOR_PEAK_TFLOPS}
            if roof_alu["frac"] > roof_hbm["frac"]:
                roof = roof_alu
        roof["kernel"] = dominant
        roof["ms_per_launch"] = per_call[dominant]
        roof["traffic"] = read_pmc_traffic(dominant, ds.name, src_hash)
        roof["algorithmic_bytes"] = traffic[dominant]

    res = {
        "metric": METRIC, "value": value, "unit": "visibilities/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ds.name, "variant": dict(VARIANT), "n_vis": m, "n": ds.n, "n_wplanes": ds.n_wplanes,
                   "support": ds.support, "beta": ds.beta, "pixel_arcsec": ds.pixel_rad / synth.ARCSEC,
                   "freq_hz": ds.freq_hz, "precision": "f32"},
        "stage_ms": per_call,
        "occupancy": {"strips_occupied": st["n_strips_occupied"],
                      "strips_total": ds.n_wplanes * ds.n // r32["info"]["strip_rows"],
                      "strip_rows": r32["info"]["strip_rows"], "planes_occupied": nw_occ},
        "roofline": roof,
        "kernel_source_hash": src_hash,
    }
    if r64 is not None:
        res["f64_value"] = m / (r64["ms_per_step"] / 1e3)
        res["f64_ms_per_step"] = r64["ms_per_step"]
        res["speedup_f32_over_f64"] = r64["ms_per_step"] / r32["ms_per_step"]
        a, b = r32["image"].astype(np.float64), r64["image"]
        res["f32_vs_f64_full_image"] = {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                                        "rel_peak": float(np.max(np.abs(a - b)) / np.max(np.abs(b)))}
        c = slice(ds.n // 2 - 256, ds.n // 2 + 256)
        res["f32_vs_f64_central_512"] = {
            "rel_l2": float(np.linalg.norm(a[c, c] - b[c, c]) / np.linalg.norm(b[c, c])),
            "rel_peak": float(np.max(np.abs(a[c, c] - b[c, c])) / np.max(np.abs(b[c, c])))}
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample of planes ...")
        res["cpu_baseline"] = cpu_baseline(ds, args.cpu_sample_planes)
    print(json.dumps(res), flush=True)


def bench_adjoint(args):
    """The differentiable-operator workload: loss + gradient per step."""
    import numpy as np
    import torch
    import synth
    import paper_2601_19714_amd as ws

    t0 = time.perf_counter()
    ds = synth.make_config(5, device="cuda" if torch.cuda.is_available() else "cpu").as_precision("f32")
    sky = synth.sky_image(ds)
    log(f"generated {ds.name}: M={ds.m} n={ds.n} nw={ds.n_wplanes} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    uvw = torch.from_numpy(ds.uvw_m).to(dev)
    V = torch.from_numpy(ds.vis).to(dev)
    w = torch.full((ds.m,), 1.0e4, dtype=torch.float32, device=dev)
    op = ws.ImagingOperator(uvw, w, ds.freq_hz, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta,
                            precision="f32")
    X = torch.tensor(sky, dtype=torch.float32, device=dev, requires_grad=True)

    def step():
        X.grad = None
        r = op(X) - V
        loss = (w * (r.real ** 2 + r.imag ** 2)).sum()
        loss.backward()
        return loss

    for _ in range(args.warmup + 1):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    # the two directions alone
    with torch.no_grad():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            y = op.predict(X.detach())
        torch.cuda.synchronize()
        ms_pred = 1e3 * (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.adjoint(y)
        torch.cuda.synchronize()
        ms_adj = 1e3 * (time.perf_counter() - t0) / args.steps
    log(f"loss+gradient: {ms:.3f} ms/step; prediction {ms_pred:.3f} ms, transpose {ms_adj:.3f} ms")
    res = {
        "metric": "visibilities/s through loss + gradient (prediction and its transpose), 1 GPU",
        "value": ds.m / (ms / 1e3), "unit": "visibilities/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c5_adjoint_f32", "n_vis": ds.m, "n": ds.n, "n_wplanes": ds.n_wplanes,
                   "support": ds.support, "precision": "f32"},
        "ms_prediction": ms_pred, "ms_transpose": ms_adj,
        "kernel_source_hash": kernel_source_hash(),
    }
    op.close()
    print(json.dumps(res), flush=True)


def bench_batch(args):
    """The batched-channel workload: aggregate and per-channel throughput."""
    import torch
    import synth

    t0 = time.perf_counter()
    chans = synth.make_channels(device="cuda" if torch.cuda.is_available() else "cpu")
    d = chans[0]
    log(f"generated {len(chans)} channels: rows {min(c.m for c in chans)}..{max(c.m for c in chans)}, "
        f"n={d.n} nw={d.n_wplanes} W={d.support} in {time.perf_counter() - t0:.1f}s")
    r = run_gpu_batch(chans, args.steps, args.warmup)
    m = sum(r["counts"])
    calls = max(1, r["timing"]["calls"])
    per_call = {k: v / calls for k, v in r["timing"]["ms"].items()}
    log(f"graph replay: {r['ms_per_step_graph']:.3f} ms/step")
    log(f"batch: {r['ms_per_step']:.3f} ms/step ({len(chans)} channels), single calls "
        f"{r['ms_per_step_single_calls']:.3f} ms; stages(ms/call) " +
        ", ".join(f"{k}={v:.4f}" for k, v in per_call.items()))
    st = r["stats"]
    m_kept = sum(s["n_gridded"] for s in st)
    n_occ = sum(s["n_strips_occupied"] for s in st)
    nw_occ = sum(s["n_planes_occupied"] for s in st)
    traffic = algorithmic_traffic("f32", d.n, m_kept, n_occ, r["info"]["strip_rows"])
    traffic["cols_stack"] += (len(chans) - 1) * d.n * d.n * 4       # one image per channel
    dominant = max(per_call, key=per_call.get)
    roof = None
    if dominant in traffic:
        gbs = traffic[dominant] / (per_call[dominant] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
        if dominant == "cols_stack":
            tf = cols_stack_flops(d.n, nw_occ) / (per_call[dominant] / 1e3) / 1e12
            if tf / FP32_VECTOR_PEAK_TFLOPS > roof["frac"]:
                roof = {"bound": "alu", "achieved": tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / FP32_VECTOR_PEAK_TFLOPS}
        roof["kernel"] = dominant
        roof["ms_per_launch"] = per_call[dominant]
        roof["traffic"] = read_pmc_traffic(dominant, "c4_batched_f32", kernel_source_hash())
        roof["algorithmic_bytes"] = traffic[dominant]
    res = {
        "metric": METRIC, "value": m / (r["ms_per_step"] / 1e3), "unit": "visibilities/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_batched_f32", "variant": dict(VARIANT), "n_channels": len(chans), "n_vis": m,
                   "rows_per_channel": [min(r["counts"]), max(r["counts"])], "n": d.n,
                   "n_wplanes": d.n_wplanes, "support": d.support, "freq_hz": [chans[0].freq_hz, chans[-1].freq_hz],
                   "precision": "f32"},
        "per_channel_ms": r["ms_per_step"] / len(chans),
        "ms_per_step_graph_replay": r["ms_per_step_graph"],
        "single_call_value": m / (r["ms_per_step_single_calls"] / 1e3),
        "batch_speedup_over_single_calls": r["ms_per_step_single_calls"] / r["ms_per_step"],
        "stage_ms": per_call,
        "occupancy": {"strips_occupied": n_occ, "planes_occupied": nw_occ},
        "roofline": roof,
        "kernel_source_hash": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample of one channel's planes ...")
        cb = cpu_baseline(chans[0], args.cpu_sample_planes)
        cb["sample"] = "channel 0 only (its per-visibility rate stands for every channel): " + cb["sample"]
        res["cpu_baseline"] = cb
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
