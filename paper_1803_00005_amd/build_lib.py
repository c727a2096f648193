"""Builds libhgf.so (the HIP kernels and the C ABI) in-tree for gfx950.

Every ``csrc/*.hip`` file, and one generated instantiation unit per
(channel count, radius) of the coefficient kernel and per channel count of
the output, guidance-statistics and one-label kernels (written to
``_build/gen/``: each holds only explicit template instantiations of the
``csrc`` headers), is compiled to an object under ``_build/`` in parallel,
then linked into ``paper_1803_00005_amd/libhgf.so``.  Packed FP32
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
GEN = os.path.join(BUILD, "gen")
# compiled set of the templated kernels (must match kMaxN / kMinRadius /
# kMaxRadius in csrc/hgf_device.hpp and csrc/hgf_launch.hpp)
CHANNELS = range(1, 20)
RADII = range(0, 10)
LIB = os.path.join(PKG, "libhgf.so")

ARCH = "gfx950"
HIPFLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}",
    f"-I{CSRC}",
]


# Sources that define each strip kernel and the launch geometry it runs with.
_COMMON = ("hgf_device.hpp", "hgf_launch.hpp", "hgf_api.hip", "runtime.hpp", "dispatch.hip")
KERNEL_SOURCES = {
    "coef_kernel": ("coef.hpp",) + _COMMON,
    "out_kernel": ("out.hpp", "out.hip") + _COMMON,
    "moments_kernel": ("guide_kernels.hpp",) + _COMMON,
    "invert_kernel": ("guide_kernels.hpp",) + _COMMON,
    "invert_lanes_kernel": ("guide_kernels.hpp",) + _COMMON,
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


def generate() -> list[str]:
    """Write the instantiation units (only those whose text changed) and
    return their paths."""
    os.makedirs(GEN, exist_ok=True)
    units = {}
    for n in CHANNELS:
        for r in RADII:
            units[f"coef_n{n}_r{r}.hip"] = (
                f'#include "coef.hpp"\n'
                f"namespace hgf {{\n"
                f"template hipError_t coef_launch_nr<{n}, {r}>(const CoefLaunch&, hipStream_t);\n"
                f"}}\n")
        units[f"out_n{n}.hip"] = (
            f'#include "out.hpp"\n'
            f"namespace hgf {{\n"
            f"template hipError_t out_launch_n<{n}>(const OutLaunch&, hipStream_t);\n"
            f"}}\n")
        units[f"guide_n{n}.hip"] = (
            f'#include "guide_kernels.hpp"\n'
            f"namespace hgf {{\n"
            f"template hipError_t moments_n<{n}>(const double*, int, int, int, int, double*,\n"
            f"                                  double, int, double*, void*, int*, hipStream_t);\n"
            f"template hipError_t invert_n<{n}>(const double*, int, int, int, double, int,\n"
            f"                                 double*, void*, hipStream_t);\n"
            f"}}\n")
        units[f"single_n{n}.hip"] = (
            f'#include "single.hpp"\n'
            f"namespace hgf {{\n"
            f"template hipError_t single_launch_n<{n}>(const SingleLaunch&, hipStream_t);\n"
            f"}}\n")
    paths = []
    for name, text in units.items():
        path = os.path.join(GEN, name)
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as fh:
                fh.write(text)
        paths.append(path)
    return sorted(paths)


def sources() -> list[str]:
    own = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    return own + generate()


def _cost(path: str) -> tuple[int, str]:
    import re
    b = os.path.basename(path)
    m = re.match(r"(coef|guide|single|out)_n(\d+)", b)
    if m is None:
        return (0, b)
    weight = {"coef": 10, "guide": 4, "single": 2, "out": 3}[m.group(1)]
    return (-weight * int(m.group(2)), b)


def _newest_dependency() -> float:
    """Modification time of the newest header or build-script change."""
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps += [os.path.join(ROOT, "include", "hgf.h"), os.path.abspath(__file__)]
    return max(os.path.getmtime(d) for d in deps)


def _compile(src: str, verbose: bool, incremental: bool = False) -> tuple[str, float]:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(src) and t > _newest_dependency():
            return obj, 0.0
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


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link the shared library; returns its path.
    ``incremental`` (development only) skips objects newer than their source
    and every header."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    # the largest units (most channels) first, so that they do not finish last
    srcs.sort(key=_cost)
    jobs = jobs or min(16, os.cpu_count() or 4, len(srcs))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, verbose, incremental): s for s in srcs}
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
    ap.add_argument("--incremental", action="store_true",
                    help="reuse objects newer than their source and every header (development)")
    a = ap.parse_args()
    t0 = time.time()
    path = build(a.jobs, a.verbose, a.incremental)
    print(f"built {path} in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
