"""Build the strip-decomposition tuning table for this GPU.

    python -m paper_1803_00005_amd.tune_table [--out PATH] [--quick]

Runs hgf_autotune on synthetic inputs of each size class the benchmarks use
(the named workloads, and images of 2^16 .. 2^21 pixels for every channel
count and radius of the batched and serving mixes, and gray guidance) and saves the table with
hgf_tune_save.  A context loads it with hgf_tune_load (Context.tune_load).
Needs a GPU.
"""
from __future__ import annotations

import argparse
import os
import sys

_PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(_PKG, "tuning_mi355x.txt")


def _shapes(quick: bool):
    from . import synth
    named = [synth.WORKLOADS[k] for k in ("rgb64_n3_L16", "voronoi450x375_n9_L60",
                                          "voronoi1242x375_n19_L128",
                                          "voronoi1242x375_n19_L128_bf16",
                                          "voronoi1242x375_n19_L128_f16")]
    if quick:
        return named
    out = []
    # size classes floor(log2 P) = 16 .. 20 for the mixes' channel counts and radii
    for cls in range(16, 21):
        P = 3 << (cls - 1)  # 1.5 * 2^cls pixels: the middle of the class
        H = int((P * 9 / 16) ** 0.5)
        W = P // H
        for degree, eps in ((1, 1e-4), (2, 1e-4), (3, 1e-3)):
            for radius in (4, 9):
                for dt in (("f32", "bf16") if degree >= 2 else ("f32",)):
                    out.append(synth.Workload(
                        name=f"class{cls}_d{degree}_r{radius}_{dt}", height=H, width=W,
                        regions=40, labels=64, radius=radius, eps=eps, degree=degree,
                        disparity="planar", seed=7000 + cls, cost_dtype=dt))
        # gray guidance, n = 1
        for radius in (4, 9):
            out.append(synth.Workload(
                name=f"class{cls}_gray_r{radius}_f32", height=H, width=W, regions=40,
                labels=64, radius=radius, eps=1e-4, degree=1, disparity="planar",
                seed=7100 + cls, guide_channels=1))
    # the named workloads last, so their own measurements decide their classes
    return out + named


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--base", default=DEFAULT_TABLE,
                    help="table to start from (its other entries are kept); 'none' starts empty")
    ap.add_argument("--quick", action="store_true", help="named workloads only")
    args = ap.parse_args()
    import torch

    from . import hgf, synth
    dev = torch.device("cuda", 0)
    ctx = hgf.Context(0)
    if args.base != "none" and os.path.exists(args.base):
        ctx.tune_load(args.base)
    for w in _shapes(args.quick):
        g, c = synth.make_workload_device(w, dev)
        # the n = 19 workloads are also run with the float64 solve (its own
        # coefficient kernel)
        for stats in (("f32", "f64") if w.n >= 10 else ("f32",)):
            ctx.autotune(g, c, radius=w.radius, eps=w.eps, degree=w.degree, basis=w.basis,
                         stats_dtype=stats)
            torch.cuda.synchronize()
        rows = [r for r in ctx.tune_entries() if r[1] == w.n and r[2] == w.radius]
        print(f"[tune] {w.name}: {len(rows)} entries", flush=True)
        del g, c
    ctx.tune_save(args.out)
    print(f"[tune] saved {len(ctx.tune_entries())} entries to {args.out}", flush=True)
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
