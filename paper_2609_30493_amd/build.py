"""Compile the HIP sources under csrc/ into libfgraft.so (gfx950).

Every source is compiled separately (in parallel) and linked into one shared
library in this package directory.  Flags:
  -ffp-contract=off   the declared float32 order relies on explicit FMAs
                      only (hipcc would otherwise fuse a*b+c by itself);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keep the compiler from emitting packed-FP32 VALU ops.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfgraft.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
ARCH = os.environ.get("FGRAFT_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _compile(src: str, defines=(), tag: str = "") -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    cmd = [hipcc(), *FLAGS, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    return obj


def build(jobs: int | None = None, defines=(), out: str | None = None) -> str:
    """Compile every source and link.  `defines` / `out` build a variant
    (e.g. FG_PROFILE, the phase-timer build) under another name."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    tag = "".join("." + d.lower() for d in defines)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, defines, tag), srcs))
    target = out or OUT
    tmp = target + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build())
