"""Builds libhgf.so (the HIP kernels and the C ABI) in-tree for gfx950.

Every ``csrc/*.hip`` file is compiled to an object under ``_build/`` (in
parallel), then linked into ``paper_1803_00005_amd/libhgf.so``.  Packed FP32
instructions are disabled for all device code.

    python -m paper_1803_00005_amd.build_lib [--jobs N] [--verbose]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhgf.so")

ARCH = "gfx950"
HIPFLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}",
]


# Sources that define each strip kernel and the launch geometry it runs with.
_COMMON = ("hgf_device.hpp", "hgf_launch.hpp", "hgf_api.hip", "runtime.hpp")
KERNEL_SOURCES = {
    "coef_kernel": ("coef.hpp", "coef_n") + _COMMON,
    "out_kernel": ("out.hpp", "out_n", "out.hip") + _COMMON,
    "moments_kernel": ("guide.hip",) + _COMMON,
    "invert_kernel": ("guide.hip",) + _COMMON,
    "invert_lanes_kernel": ("guide.hip",) + _COMMON,
}


def source_hash(kernel: str | None = None) -> str:
    """Short hash of the kernel sources (identifies the code a measurement was
    taken on): all of them, or the files that define one kernel."""
    import hashlib
    h = hashlib.sha256()
    prefixes = KERNEL_SOURCES.get(kernel) if kernel else None
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".hpp")):
            continue
        if prefixes is not None and not any(f == p or f.startswith(p) for p in prefixes):
            continue
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HGF library needs ROCm's hipcc to build")


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, verbose: bool) -> tuple[str, float]:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [_hipcc(), *HIPFLAGS, "-c", src, "-o", obj]
    t0 = time.time()
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{proc.stdout}\n{proc.stderr}")
    if verbose and proc.stderr.strip():
        print(proc.stderr, file=sys.stderr)
    return obj, time.time() - t0


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, os.cpu_count() or 4, len(srcs))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, verbose): s for s in srcs}
        for f in cf.as_completed(futs):
            obj, dt = f.result()
            objs.append(obj)
            if verbose:
                print(f"  {os.path.basename(obj)}: {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *sorted(objs)]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"linking libhgf.so failed:\n{proc.stdout}\n{proc.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args()
    t0 = time.time()
    path = build(a.jobs, a.verbose)
    print(f"built {path} in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
