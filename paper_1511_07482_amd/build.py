"""Build libkdefft.so (HIP, gfx950) in the package directory.

Each translation unit under csrc/ is compiled by hipcc in parallel into
_build/, then linked into paper_1511_07482_amd/libkdefft.so.  Always
rebuilds every unit whose source or headers are newer than its object.

    python -m paper_1511_07482_amd.build [--jobs N] [--force]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libkdefft.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("KDEFFT_ARCH", "gfx950")

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-Wno-unused-command-line-argument",
]
# host-side arithmetic must round exactly like the CPU reference
HOST_EXTRA = ["-ffp-contract=off"]

UNITS = ["api.cpp", "noalloc.hip", "minimize.hip", "fft.hip", "bin.hip", "plain.hip", "rows.hip",
         "rows_d1.hip", "rows_d2.hip", "rows_d3.hip", "rows_d4.hip",
         "rows_eta_d1.hip", "rows_eta_d2.hip", "rows_eta_d3.hip", "rows_eta_d4.hip"]
HEADERS = ["dev_common.h", "dev_kernels.h", "eta_fun.h", "finish.h", "internal.h", "params.h", "rows_impl.h",
           "rows_dispatch.h"]


def _newest_header():
    paths = [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "kdefft.h")]
    return max(os.path.getmtime(p) for p in paths)


def _compile(unit, force):
    src = os.path.join(CSRC, unit)
    obj = os.path.join(BUILD, unit + ".o")
    if not force and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(src), _newest_header()):
            return unit, 0, "up to date"
    cmd = [HIPCC] + COMMON + (HOST_EXTRA if unit.endswith(".cpp") else []) + ["-x", "hip", "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    return unit, p.returncode, (p.stdout + p.stderr)


def build(jobs=None, force=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 4)
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for unit, rc, out in ex.map(lambda u: _compile(u, force), UNITS):
            if rc != 0:
                failed.append((unit, out))
            elif verbose and out.strip() and out != "up to date":
                print(f"[{unit}]\n{out}", file=sys.stderr)
    if failed:
        for unit, out in failed:
            print(f"=== {unit} failed ===\n{out}", file=sys.stderr)
        raise RuntimeError("HIP compilation failed: " + ", ".join(u for u, _ in failed))
    objs = [os.path.join(BUILD, u + ".o") for u in UNITS]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.force, a.verbose))
