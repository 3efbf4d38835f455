"""Build-time autotuner for the kernels' shape macros.

The work-group shapes of the kernels are compile-time constants (the FFT base radix of each
pass, the pixels of a stacking block, the cells of a gridding strip, the registers the
gridding run sums may take, the stacking prefetch, ...), each a WSIMG_* macro with a default
in csrc/kernels.hpp.  This tool compiles a set of candidate macro settings and times each on
the GPU on synthetic workloads, then records the fastest in tuned.json, which build.py adds
to its hipcc line.

  python -m paper_2601_19714_amd.tune build [--out DIR] [--workloads c2,c3,c4] [--only a,b]
                                                                        (CPU: compile)
  python -m paper_2601_19714_amd.tune time [--dir DIR] [--workloads c2,c3,c4] [--steps K]
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

# name -> extra macro definitions (the empty set is the source defaults).  A candidate whose
# flags hold "{L}" is per-shape: it is built and judged separately for each image size of the
# timed workloads (L = log2 of the image side), and the fastest per-shape candidate of each size
# is kept for that size only.  The others are global: kept when their geometric-mean time over
# all workloads beats the defaults.
CANDIDATES = {
    "defaults": [],
    "stack_r8": ["-DWSIMG_F32_LR2_N{L}=3"],
    "stack_r16": ["-DWSIMG_F32_LR2_N{L}=4"],
    "strip_rows1": ["-DWSIMG_STRIP_ROWS_N{L}=1"],
    "strip_rows4": ["-DWSIMG_STRIP_ROWS_N{L}=4"],
    "chunk32": ["-DWSIMG_F32_GRID_CHUNK_MAX=32"],
    "chunk128": ["-DWSIMG_F32_GRID_CHUNK_MAX=128"],
    "walk128": ["-DWSIMG_WALK_VGPRS=128"],
}
# the image sizes (log2 n) where a per-shape candidate differs from the defaults (radix 16
# stacking at 4096^2 and radix 8 elsewhere; two-row strips below 4096^2)
APPLIES = {
    "stack_r8": lambda L: L == 12,
    "stack_r16": lambda L: L >= 10 and L != 12,
    "strip_rows1": lambda L: L < 12,
    "strip_rows4": lambda L: L < 12,
}

WORKLOADS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}
# log2 of each workload's image side (the tuned float32 path)
WORKLOAD_LOG2N = {"c1": 8, "c2": 12, "c3": 13, "c4": 10, "c5": 11}
# a candidate replaces the defaults only when its time is this much lower (two identical builds
# timed 1% apart on the 8192^2 image)
NOISE = 0.02


def per_shape(name: str) -> bool:
    return any("{L}" in f for f in CANDIDATES[name])


def variants(workloads):
    """(library name, candidate, log2 n or None, flags) for every library to build."""
    out = []
    shapes = sorted({WORKLOAD_LOG2N[w] for w in workloads})
    for name, flags in CANDIDATES.items():
        if per_shape(name):
            for L in shapes:
                if APPLIES.get(name, lambda _: True)(L):
                    out.append((f"{name}_n{L}", name, L, [f.replace("{L}", str(L)) for f in flags]))
        else:
            out.append((name, name, None, list(flags)))
    return out


def build_all(out: str, workloads, names=None):
    from . import build as _build
    os.makedirs(out, exist_ok=True)
    procs = []
    for lib_name, name, _, flags in variants(workloads):
        if names and name not in names:
            continue
        lib = os.path.join(out, f"libwsimg_{lib_name}.so")
        cmd = [_build.hipcc()] + _build.flags() + flags + [_build.SRC, "-o", lib]
        procs.append((lib_name, subprocess.Popen(cmd, stderr=subprocess.DEVNULL)))
    failed = [n for n, p in procs if p.wait() != 0]
    for n, _ in procs:
        print(f"{n}: {'FAILED' if n in failed else 'ok'}", flush=True)
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


def _run_child(lib: str, wl: str, steps: int, warmup: int, timeout: int) -> float:
    cmd = [sys.executable, "-m", "paper_2601_19714_amd.tune", "_run", "--lib", lib, "--workload", wl,
           "--steps", str(steps), "--warmup", str(warmup)]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0:
        print(f"{os.path.basename(lib)} {wl}: failed (exit {r.returncode}); stopping", flush=True)
        print(r.stderr[-2000:], flush=True)
        raise SystemExit(r.returncode or 1)
    return json.loads(r.stdout.strip().splitlines()[-1])["ms"]


def time_all(src: str, workloads, steps: int, warmup: int, timeout: int):
    """Time every built variant on the workloads it applies to; choose per shape and globally."""
    results = {}            # library name -> workload -> ms
    for lib_name, name, L, _ in variants(workloads):
        lib = os.path.join(src, f"libwsimg_{lib_name}.so")
        if not os.path.exists(lib):
            print(f"{lib_name}: not built, skipped", flush=True)
            continue
        results[lib_name] = {}
        for wl in workloads:
            if L is not None and WORKLOAD_LOG2N[wl] != L:
                continue
            results[lib_name][wl] = ms = _run_child(lib, wl, steps, warmup, timeout)
            print(f"{lib_name} {wl}: {ms:.3f} ms", flush=True)
    base = results.get("defaults")
    if not base:
        raise SystemExit("the defaults library was not timed")
    flags, chosen = [], {}
    # per shape: the fastest per-shape candidate of each size (summed over that size's workloads)
    for L in sorted({WORKLOAD_LOG2N[w] for w in workloads}):
        wls = [w for w in workloads if WORKLOAD_LOG2N[w] == L]
        t0 = sum(base[w] for w in wls)
        best, tbest = "defaults", t0
        for lib_name, name, LL, fl in variants(workloads):
            if LL == L and lib_name in results and all(w in results[lib_name] for w in wls):
                t = sum(results[lib_name][w] for w in wls)
                if t < tbest * (1.0 - NOISE) and t < t0 * (1.0 - NOISE):
                    best, tbest = lib_name, t
        entry = {"candidate": best, "ms": tbest, "defaults_ms": t0, "workloads": wls, "flags": []}
        if best != "defaults":
            entry["flags"] = next(fl for ln, _, _, fl in variants(workloads) if ln == best)
            flags += entry["flags"]
        chosen[f"f32/{L}"] = entry
    # global: geometric mean over all workloads
    score = {}
    for lib_name, name, L, _ in variants(workloads):
        res = results.get(lib_name, {})
        if L is None and len(res) == len(workloads):
            score[lib_name] = math.exp(sum(math.log(res[wl] / base[wl]) for wl in workloads) / len(workloads))
    gbest = min(score, key=score.get)
    if score[gbest] > 1.0 - NOISE:        # within timing noise of the source defaults: keep them
        gbest = "defaults"
    flags += CANDIDATES[gbest]
    rec = {"flags": flags, "per_shape": chosen, "global": {"candidate": gbest, "score_vs_defaults": score},
           "ms": results, "workloads": list(workloads), "steps": steps}
    with open(TUNED, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"per shape: { {k: v['candidate'] for k, v in chosen.items()} }; global: {gbest}; "
          f"flags {flags}; written to {TUNED}", flush=True)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--out", default=DEFAULT_DIR)
    b.add_argument("--workloads", default="c1,c2,c3,c4")
    b.add_argument("--only", default="", help="comma-separated candidate names (default: all)")
    t = sub.add_parser("time")
    t.add_argument("--dir", default=DEFAULT_DIR)
    t.add_argument("--workloads", default="c1,c2,c3,c4")
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
        wls = [w for w in a.workloads.split(",") if w]
        only = [x for x in a.only.split(",") if x] or None
        sys.exit(1 if build_all(a.out, wls, only) else 0)
    if a.cmd == "time":
        time_all(a.dir, [w for w in a.workloads.split(",") if w], a.steps, a.warmup, a.timeout)
    if a.cmd == "_run":
        _time_one(a.lib, a.workload, a.steps, a.warmup)


if __name__ == "__main__":
    main()
