"""Build-time autotuner for the kernels' shape macros.

The work-group shapes of the kernels are compile-time constants (the FFT base radix of each
pass, the pixels of a stacking block, the cells of a gridding strip, the registers the
gridding run sums may take, the stacking prefetch, ...), each a WSIMG_* macro with a default
in csrc/kernels.hpp.  This tool compiles a set of candidate macro settings and times each on
the GPU on synthetic workloads, then records the fastest in tuned.json, which build.py adds
to its hipcc line.

  python -m paper_2601_19714_amd.tune build [--out DIR]                 (CPU: compile)
  python -m paper_2601_19714_amd.tune time [--dir DIR] [--workloads c2,c4] [--steps K]
                                                                        (GPU: time, write tuned.json)
Each candidate is timed in a child process of its own (one library per process).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TUNED = os.path.join(HERE, "tuned.json")
DEFAULT_DIR = os.path.join(HERE, "_tune")

# name -> extra macro definitions (the empty set is the source defaults)
CANDIDATES = {
    "defaults": [],
    "stack_r8": ["-DWSIMG_F32_LR2=3"],
    "stack_b2": ["-DWSIMG_F32_BS=0", "-DWSIMG_F32_LR2=3"],
    "strip_rows_by_cells": ["-DWSIMG_STRIP_ROWS_SMALL=0"],
    "chunk32": ["-DWSIMG_GRID_CHUNK_MAX=32"],
    "tw_table": ["-DWSIMG_TW_DERIVE=0"],
    "walk128": ["-DWSIMG_WALK_VGPRS=128"],
}

WORKLOADS = {"c1": 1, "c2": 2, "c4": 4, "c5": 5}
# a candidate replaces the defaults only when its geometric-mean time is this much lower
NOISE = 0.01


def build_all(out: str, names=None):
    from . import build as _build
    os.makedirs(out, exist_ok=True)
    procs = []
    for name in names or CANDIDATES:
        lib = os.path.join(out, f"libwsimg_{name}.so")
        cmd = [_build.hipcc()] + _build.flags() + CANDIDATES[name] + [_build.SRC, "-o", lib]
        procs.append((name, subprocess.Popen(cmd, stderr=subprocess.DEVNULL)))
    failed = [name for name, p in procs if p.wait() != 0]
    for name, _ in procs:
        print(f"{name}: {'FAILED' if name in failed else 'ok'}", flush=True)
    return failed


def _time_one(lib: str, workload: str, steps: int, warmup: int):
    """Child process body: the imaging call of one workload with library `lib`, ms per call."""
    import torch
    torch.cuda.init()
    from . import _lib
    _lib.load(lib)
    import paper_2601_19714_amd as ws
    sys.path.insert(0, ROOT)
    import synth
    dev = torch.device("cuda:0")
    cfg = WORKLOADS[workload]
    if cfg == 4:
        chans = synth.make_channels(device="cuda")
        uvw, vis, wts, counts, freqs = synth.stack_channels(chans)
        d = chans[0]
        u, v, w = (torch.from_numpy(a).to(dev) for a in (uvw, vis, wts))
        plan = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, "f32", max_vis=len(wts),
                       max_channels=len(counts))

        def call():
            plan.image_batch(u, v, w, counts, freqs)
    elif cfg == 5:
        d = synth.make_config(5, device="cuda").as_precision("f32")
        u, w = torch.from_numpy(d.uvw_m).to(dev), torch.from_numpy(d.weights).to(dev)
        img = torch.from_numpy(synth.sky_image(d).astype("float32")).to(dev)
        plan = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, "f32", max_vis=d.m)

        def call():
            plan.predict(u, w, d.freq_hz, img)
    else:
        d = synth.make_config(cfg, device="cuda").as_precision("f32")
        u, v, w = (torch.from_numpy(a).to(dev) for a in (d.uvw_m, d.vis, d.weights))
        plan = ws.Plan(d.n, d.pixel_rad, d.n_wplanes, d.support, d.beta, "f32", max_vis=d.m)

        def call():
            plan.image(u, v, w, d.freq_hz)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    print(json.dumps({"ms": 1e3 * (time.perf_counter() - t0) / steps}), flush=True)


def time_all(src: str, workloads, steps: int, warmup: int, timeout: int):
    results = {}
    for name in CANDIDATES:
        lib = os.path.join(src, f"libwsimg_{name}.so")
        if not os.path.exists(lib):
            print(f"{name}: not built, skipped", flush=True)
            continue
        results[name] = {}
        for wl in workloads:
            cmd = [sys.executable, "-m", "paper_2601_19714_amd.tune", "_run", "--lib", lib, "--workload", wl,
                   "--steps", str(steps), "--warmup", str(warmup)]
            r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=timeout)
            if r.returncode != 0:
                print(f"{name} {wl}: failed (exit {r.returncode}); stopping", flush=True)
                print(r.stderr[-2000:], flush=True)
                raise SystemExit(r.returncode or 1)
            ms = json.loads(r.stdout.strip().splitlines()[-1])["ms"]
            results[name][wl] = ms
            print(f"{name} {wl}: {ms:.3f} ms", flush=True)
    base = results.get("defaults")
    score = {}
    for name, res in results.items():
        if len(res) == len(workloads) and base:
            score[name] = math.exp(sum(math.log(res[wl] / base[wl]) for wl in workloads) / len(workloads))
    best = min(score, key=score.get)
    if score[best] > 1.0 - NOISE:        # within timing noise of the source defaults: keep them
        best = "defaults"
    rec = {"flags": CANDIDATES[best], "candidate": best, "score_vs_defaults": score,
           "ms": results, "workloads": list(workloads), "steps": steps}
    with open(TUNED, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"best: {best} ({score[best]:.3f} of the defaults' time); written to {TUNED}", flush=True)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--out", default=DEFAULT_DIR)
    t = sub.add_parser("time")
    t.add_argument("--dir", default=DEFAULT_DIR)
    t.add_argument("--workloads", default="c2,c4")
    t.add_argument("--steps", type=int, default=10)
    t.add_argument("--warmup", type=int, default=2)
    t.add_argument("--timeout", type=int, default=240)
    r = sub.add_parser("_run")
    r.add_argument("--lib", required=True)
    r.add_argument("--workload", required=True)
    r.add_argument("--steps", type=int, default=10)
    r.add_argument("--warmup", type=int, default=2)
    a = ap.parse_args(argv)
    if a.cmd == "build":
        sys.exit(1 if build_all(a.out) else 0)
    if a.cmd == "time":
        time_all(a.dir, [w for w in a.workloads.split(",") if w], a.steps, a.warmup, a.timeout)
    if a.cmd == "_run":
        _time_one(a.lib, a.workload, a.steps, a.warmup)


if __name__ == "__main__":
    main()
