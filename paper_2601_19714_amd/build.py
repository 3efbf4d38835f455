"""Compile the HIP library (libwsimg.so) in-tree for gfx950 with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "wsimg.hip")
LIB = os.path.join(HERE, "libwsimg.so")
DEPS = [os.path.join(HERE, "csrc", f) for f in
        ("wsimg.hip", "kernels.hpp", "fft_lds.hpp", "device_common.hpp", "host_tables.hpp")] + \
       [os.path.join(ROOT, "include", "wsimg.h")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(arch: str = "gfx950"):
    return [
        f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed fp32 instructions stay off in all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fno-gpu-rdc", "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"),
    ]


def tuned_flags():
    """Macro definitions recorded by the autotuner (paper_2601_19714_amd/tune.py), if it ran."""
    path = os.path.join(HERE, "tuned.json")
    if not os.path.exists(path):
        return []
    import json
    with open(path) as fh:
        return list(json.load(fh).get("flags", []))


def build(verbose: bool = False, extra=()) -> str:
    """Compile libwsimg.so; the macro settings recorded by the autotuner (tuned.json), if any,
    come first, then `extra`."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + flags() + tuned_flags() + list(extra) + [SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
