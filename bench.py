#!/usr/bin/env python3
"""Throughput of the w-stacking imager on one MI355X: visibilities imaged per second.

A step is one whole dirty image (all stages: bucket sort, gridding + row FFT, column
FFT + w-phase + stacking + taper) of one synthetic visibility set already resident in HBM.
The default workload is the largest single-GPU one, LOFAR-shaped: 2^26 visibilities from 60
stations spread log-radially to 100 km, 150 MHz, 8192^2 image, 64 w-planes, Kaiser-Bessel
support 9, float32 path; the float64 path is timed on the same inputs and its rate and the
float32/float64 speedup are reported too.  --workload c2 selects the MeerKAT-shaped single
channel (7 257 600 visibilities, 4096^2, 32 w-planes, support 7).

Both benched images are compared with the float64 oracle (vs_oracle): over every pixel on
the support-7 workloads, at 32 x 32 pixels spread over the central 512^2 crop on the
LOFAR-shaped one (where the oracle's cost is its gridding of all rows).

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
  roofline_gridding : the gridding stage (prep, sort, gridding + row transform) against the
                 HBM peak: input rows plus row-transformed occupied strips over its time;
  cpu_baseline : the FP64 oracle timed on the same workload on the host cores (all the cores
                 this process may use, at most 16), the whole image where that takes a few
                 tens of seconds, else a stated sample of w-planes (test infrastructure, run
                 only here, rank 0, N = 1).
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


def host_threads(cap: int = 16) -> int:
    """Cores this process may run on (sched_getaffinity), at most cap: a GPU machine gives one
    GPU's share of its cores to the job."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _errs(a, ref):
    import numpy as np
    d = a.astype(np.float64) - ref
    return {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "rel_peak": float(np.max(np.abs(d)) / np.max(np.abs(ref)))}


def oracle_check(ds, images: dict):
    """The benched images against the float64 oracle.  Support 7: every pixel (and the inner
    half); support 9: 32 x 32 pixels spread over the central 512^2 crop.  Returns the errors
    and, where the oracle made the whole image, its wall time (it doubles as cpu_baseline)."""
    import numpy as np
    import oracle
    d = ds.as_precision("f64")
    prm = oracle.Params(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, **_oracle_variant())
    th = host_threads()
    out = {"threads": th}
    t0 = time.perf_counter()
    if d.support <= 7:
        ref = oracle.wstack_image(d.uvw_m, d.vis, d.weights, d.freq_hz, prm, threads=th)
        wall = time.perf_counter() - t0
        q = slice(d.n // 4, 3 * d.n // 4)
        for prec, img in images.items():
            out[prec] = {"full_image": _errs(img, ref), "inner_half": _errs(img[q, q], ref[q, q])}
        out["where"] = "every pixel"
        out["oracle_whole_image_s"] = wall
    else:
        rng = np.random.default_rng(3)
        lo = d.n // 2 - 256
        rows = np.unique(np.concatenate([[d.n // 2], rng.choice(np.arange(lo, lo + 512), 31, replace=False)]))
        cols = np.unique(np.concatenate([[d.n // 2], rng.choice(np.arange(lo, lo + 512), 31, replace=False)]))
        ref = oracle.wstack_image(d.uvw_m, d.vis, d.weights, d.freq_hz, prm, pixels=(rows, cols), threads=th)
        for prec, img in images.items():
            out[prec] = {"crop_sampled": _errs(img[np.ix_(rows, cols)], ref)}
        out["where"] = f"{rows.size} x {cols.size} pixels of the central 512^2 crop"
        out["oracle_s"] = time.perf_counter() - t0
    ok = True
    for prec in images:
        tol = 1e-5 if prec == "f32" else 1e-12
        ok &= all(v <= tol for part in out[prec].values() for v in part.values())
    out["within_tolerance"] = bool(ok)
    return out


def _oracle_variant():
    v = {}
    if VARIANT.get("fold_w"):
        v["fold"] = True
    if VARIANT.get("pad") == 2:
        v["pad"] = 2
    return v


def cpu_baseline(ds, check=None):
    """The oracle's imaging rate on the host cores: the whole-image time of the oracle check
    when it made the whole image, else the oracle on every 4th w-plane (all rows of those
    planes, whole image), scaled to all planes: M / (T_prepare + 4 T_sampled)."""
    import oracle
    th = host_threads()
    d = ds.as_precision("f64")
    if check is not None and "oracle_whole_image_s" in check:
        wall = check["oracle_whole_image_s"]
        return {"value": d.m / wall, "unit": "visibilities/s", "cores": check["threads"], "kind": "oracle",
                "sample": (f"whole image, all {d.m} rows, every step of the FP64 oracle (C gridding loop, "
                           f"numpy FFT, w-phase, stack, taper), w-planes in {check['threads']} threads: "
                           f"{wall:.1f} s")}
    prm = oracle.Params(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, **_oracle_variant())
    t0 = time.perf_counter()
    pr = oracle.prepare(d.uvw_m, d.weights, d.freq_hz, prm)
    t_prep = time.perf_counter() - t0
    step = 4 if d.n_wplanes >= 8 else 1
    planes = list(range(step // 2, d.n_wplanes, step))
    t0 = time.perf_counter()
    oracle.wstack_image(d.uvw_m, d.vis, d.weights, d.freq_hz, prm, planes=planes, prepared=pr, threads=th)
    t_planes = time.perf_counter() - t0
    import numpy as np
    m_sample = int(np.isin(pr.k[pr.keep], planes).sum())
    est = t_prep + (d.n_wplanes / len(planes)) * t_planes
    return {"value": d.m / est, "unit": "visibilities/s", "cores": min(th, len(planes)), "kind": "oracle",
            "sample": (f"FP64 oracle, steps 1-3 on all {d.m} rows ({t_prep:.1f} s), steps 4-8 (whole image) "
                       f"on {len(planes)} of {d.n_wplanes} w-planes (every {step}th; {m_sample} rows) in "
                       f"{min(th, len(planes))} threads ({t_planes:.1f} s); whole-image time estimated as "
                       f"prepare + {d.n_wplanes // len(planes)} x sampled = {est:.1f} s")}


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
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c3")
    ap.add_argument("--max-rows", type=int, default=None, help="a shorter track (first rows, time-major)")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 path")
    ap.add_argument("--fold", action="store_true", help="w-folding (accuracy variant)")
    ap.add_argument("--pad2", action="store_true", help="grid of twice the image side (accuracy variant)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    ds = synth.make_config(cfg, device="cuda" if torch.cuda.is_available() else "cpu", max_rows=args.max_rows)
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
    # the gridding stage (S1-S3 with the fused row transform): input rows in, occupied strips out
    grid_stages = ("zero_counts", "reduce", "key", "scan", "scatter", "origin_sort", "grid_rows")
    t_grid = sum(per_call[k] for k in grid_stages) / 1e3
    grid_bytes = m * (24 + 8 + 4) + st["n_strips_occupied"] * r32["info"]["strip_rows"] * ds.n * 8
    roof_grid = {"bound": "hbm", "achieved": grid_bytes / t_grid / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": grid_bytes / t_grid / 1e9 / HBM_PEAK_GBS, "stages": list(grid_stages),
                 "ms": t_grid * 1e3, "algorithmic_bytes": grid_bytes,
                 "bytes_rule": "36 B per input row (uvw, vis, weight) + 8 B per cell of the occupied strips"}

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
        "roofline_gridding": roof_grid,
        "kernel_source_hash": src_hash,
    }
    images = {"f32": r32["image"]}
    if r64 is not None:
        res["f64_value"] = m / (r64["ms_per_step"] / 1e3)
        res["f64_ms_per_step"] = r64["ms_per_step"]
        res["speedup_f32_over_f64"] = r64["ms_per_step"] / r32["ms_per_step"]
        res["f64_stage_ms"] = {k: v / max(1, r64["timing"]["calls"]) for k, v in r64["timing"]["ms"].items()}
        a, b = r32["image"].astype(np.float64), r64["image"]
        res["f32_vs_f64_full_image"] = _errs(a, b)
        c = slice(ds.n // 2 - 256, ds.n // 2 + 256)
        res["f32_vs_f64_central_512"] = _errs(a[c, c], b[c, c])
        images["f64"] = r64["image"]
    check = None
    if not args.no_oracle_check:
        log(f"checking the benched images against the FP64 oracle on {host_threads()} threads ...")
        check = oracle_check(ds, images)
        res["vs_oracle"] = check
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle ...")
        res["cpu_baseline"] = cpu_baseline(ds, check)
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
        cb = cpu_baseline(chans[0])
        cb["sample"] = "channel 0 only (its per-visibility rate stands for every channel): " + cb["sample"]
        res["cpu_baseline"] = cb
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
