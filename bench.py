"""Throughput of the HGF cost-volume filter on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step is one pass of the whole hot path over one synthetic cost volume that
is already resident in HBM: guidance synthesis, guidance window statistics,
per-pixel inverse, per-label coefficient box sums and solve, coefficient box
filter and output, winner-takes-all labels (one hgf_filter call).  The default
workload is the 450 x 375 colour Voronoi image with degree-2 polynomial
guidance (n = 9), 60 labels, r = 9, eps = 1e-4.

Prints one JSON line: throughput in Mpixel.labels/s, the per-stage kernel
times measured with HIP events on the filter's stream over the timed
region, the roofline position of the dominant kernel, the error of the
filtered costs against the FP64 oracle at sampled pixels, and the oracle's
own throughput on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1803_00005_amd import synth  # noqa: E402

METRIC = "filtered Mpixel·labels/s (n=9,19) at stated error vs FP64; HBM GB/s; p99"
UNIT = "Mpixel·labels/s"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
# FMA rate of the vector ALU without packed FP32: 256 CU x 4 SIMD x 16 lanes x
# 2 flop x 2.4 GHz; float64 FMAs issue at the same rate on this chip.
VALU_PEAK_TFLOPS = 78.6
DEFAULT_WORKLOAD = "voronoi450x375_n9_L60"
STAGES = ["guide_mean", "guide_synth", "guide_moments", "guide_invert", "coef", "out_wta",
          "wta_keys"]
KERNEL_NAMES = {"coef": "coef_kernel", "out_wta": "out_kernel", "guide_moments": "moments_kernel",
                "guide_invert": "invert_kernel"}


# ----------------------------------------------------------------------------
# algorithmic work per stage (bytes that must cross HBM, flops of the method)
# ----------------------------------------------------------------------------

def stage_model(w: synth.Workload, reg: str = "covariance"):
    n = w.n
    P = w.pixels
    L = w.labels
    PL = P * L
    D = n + 1 if reg == "ridge" else n
    PD = D * (D + 1) // 2
    K = n + n * (n + 1) // 2
    esz = 2 if w.cost_dtype == "bf16" else 4
    m = w.guide_channels
    return {
        # window sums of the n + 1 products (n mults, 4 running-sum adds per channel),
        # covariance 3n, product M c 2n^2, intercept 2n + 1
        "coef": dict(flops=PL * (2 * n * n + 10 * n + 5),
                     bytes=PL * (esz + 4 * (n + 1)) + P * (8 * PD + 8 * n + 4 * (n + 1))),
        # window sums of the n + 1 coefficients (4 adds each), dot with G (2n), mean (2)
        "out_wta": dict(flops=PL * (4 * (n + 1) + 2 * n + 2),
                        bytes=PL * (4 * (n + 1) + 4) + P * (4 * (n + 1) + 8)),
        "guide_moments": dict(flops=P * K * 6, bytes=P * (8 * n + 8 * K)),
        "guide_invert": dict(flops=P * (D ** 3), bytes=P * (8 * K + 8 * PD + 8 * n)),
        "guide_synth": dict(flops=P * n * 3, bytes=P * (4 * m + 8 * n + 4 * (n + 1))),
        "guide_mean": dict(flops=P * n * 3, bytes=P * 4 * m),
        "wta_keys": dict(flops=0, bytes=P * 8 * 3 + P * 4),
    }


def roofline_of(name, model, ms_per_launch, traffic):
    flops, nbytes = model["flops"], model["bytes"]
    ridge = VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if nbytes > 0 and flops / nbytes < ridge:
        achieved = nbytes / (ms_per_launch * 1e-3) / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes": nbytes, "algorithmic_flops": flops}
    achieved = flops / (ms_per_launch * 1e-3) / 1e12
    return {"kernel": name, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS, "traffic": traffic,
            "algorithmic_bytes": nbytes, "algorithmic_flops": flops}


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_00005_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, stage: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(KERNEL_NAMES.get(stage, ""), None)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


# ----------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample, on the host cores
# ----------------------------------------------------------------------------

def _oracle_crop(args):
    from threadpoolctl import threadpool_limits

    from oracle import hgf_oracle as O
    guide, cost, w = args
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.filter_covariance(O.guidance(guide, w.degree, w.basis), cost, w.radius, w.eps)
        return time.perf_counter() - t0


def cpu_baseline(w: synth.Workload, guide, cost, target_s: float = 12.0):
    import multiprocessing as mp

    cores = min(16, len(os.sched_getaffinity(0)))
    W_ = w.width
    rows = max(2 * w.radius + 2, 24)
    # calibrate on one crop, then size the sample so that every core works ~target_s
    t1 = _oracle_crop((guide[:, :rows], cost[:rows], w))
    crops_per_core = max(1, int(target_s / max(t1, 1e-3)))
    ncrops = cores * crops_per_core
    starts = [(i * rows) % max(1, w.height - rows + 1) for i in range(ncrops)]
    jobs = [(guide[:, s:s + rows], cost[s:s + rows], w) for s in starts]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_crop, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    pl = ncrops * rows * W_ * w.labels
    return {"value": pl / wall / 1e6, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"{ncrops} crops of {W_}x{rows} px x {w.labels} labels (each filtered as "
                      f"its own image, FP64 numpy, per-pixel LU), {cores} processes, "
                      f"{wall:.1f} s wall; one crop on one core: {t1:.2f} s",
            "single_core_value": rows * W_ * w.labels / t1 / 1e6}


# ----------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(synth.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the filter shards by labels or image strips; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    w = synth.WORKLOADS[args.workload]
    print(f"[bench] workload {w.name}: {w.height}x{w.width} n={w.n} L={w.labels} r={w.radius} "
          f"eps={w.eps} cost={w.cost_dtype}", file=sys.stderr, flush=True)
    guide, cost = synth.make_workload(w)

    # the host-core oracle runs before the GPU is touched (forked workers)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, guide, cost)
        print(f"[bench] cpu baseline {cpu['value']:.3f} {UNIT} on {cpu['cores']} cores",
              file=sys.stderr, flush=True)

    import torch

    from paper_1803_00005_amd import hgf

    dev = torch.device("cuda", 0)
    g_d = torch.from_numpy(guide).to(dev)
    c_d = torch.from_numpy(cost).to(dev)
    if w.cost_dtype == "bf16":
        c_d = c_d.to(torch.bfloat16)
    ctx = hgf.Context(0)
    p = hgf.make_params(w.height, w.width, w.labels, radius=w.radius, eps=w.eps, degree=w.degree,
                        guide_channels=w.guide_channels, basis=w.basis, cost_dtype=w.cost_dtype)
    ws = torch.empty(hgf.workspace_size(p), dtype=torch.uint8, device=dev)
    Z = torch.empty((w.height, w.width, w.labels), dtype=torch.float32, device=dev)
    lab = torch.empty((w.height, w.width), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        ctx.filter(g_d, c_d, radius=w.radius, eps=w.eps, degree=w.degree, basis=w.basis,
                   out=Z, labels=lab, workspace=ws, stream=stream)

    if args.copy_calibration:
        # a fill (writes 1 GiB) and a sum (reads 1 GiB): known byte counts for
        # the HBM byte counters
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        for _ in range(3):
            s_ = src.sum()
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: fill and 3 sums of {src.numel() * 4} bytes "
              f"(sum={float(s_):.0f})", file=sys.stderr, flush=True)
        del src

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    if not args.no_stage_timing:
        ctx.set_stage_timing(True)
        ctx.stage_times()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    stages = ctx.stage_times() if not args.no_stage_timing else {}
    ctx.set_stage_timing(False)
    print(f"[bench] timed {args.steps} steps: {ms:.4f} ms/step (wall {wall:.3f} s)",
          file=sys.stderr, flush=True)

    value = w.pixel_labels / (ms * 1e-3) / 1e6
    model = stage_model(w)
    stage_rows = []
    for name in STAGES:
        if name not in stages:
            continue
        tot, cnt = stages[name]
        if cnt == 0:
            continue
        per = tot / cnt
        launches_per_step = cnt / args.steps
        mdl = {k: v / launches_per_step for k, v in model[name].items()}
        rf = roofline_of(name, mdl, per, None)
        stage_rows.append({"stage": name, "ms_per_step": tot / args.steps, "launches": cnt,
                           "ms_per_launch": per, "bound": rf["bound"],
                           "achieved": round(rf["achieved"], 3), "unit": rf["unit"],
                           "frac": round(rf["frac"], 4)})
    roof = None
    if stage_rows:
        dom = max(stage_rows, key=lambda r: r["ms_per_step"])
        cnt = stages[dom["stage"]][1]
        mdl = {k: v / (cnt / args.steps) for k, v in model[dom["stage"]].items()}
        roof = roofline_of(KERNEL_NAMES.get(dom["stage"], dom["stage"]), mdl,
                           dom["ms_per_launch"], measured_traffic(w.name, dom["stage"]))

    err = None
    if not args.no_check:
        from oracle import hgf_oracle as O
        Zh = Z.cpu().numpy().astype(np.float64)
        lh = lab.cpu().numpy()
        rng = np.random.default_rng(0)
        pts = sorted({(0, 0), (w.height - 1, w.width - 1)} |
                     {(int(rng.integers(0, w.height)), int(rng.integers(0, w.width)))
                      for _ in range(14)})
        idx = tuple(np.array(pts).T)
        Zo = O.filter_points(O.guidance(guide, w.degree, w.basis), cost, w.radius, w.eps, pts)
        scale = np.maximum(np.abs(Zo), np.abs(cost).max())
        rel = float(np.max(np.abs(Zh[idx] - Zo) / scale))
        agree = bool(np.all((lh[idx] == O.wta(Zo)) | O.near_tie_mask(Zo)))
        err = {"max_rel_vs_fp64_oracle": rel, "tolerance": 1e-4, "points": len(pts),
               "labels_agree_outside_near_ties": agree}

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "height": w.height, "width": w.width, "labels": w.labels,
                   "n": w.n, "degree": w.degree, "basis": w.basis, "radius": w.radius,
                   "eps": w.eps, "cost_dtype": w.cost_dtype, "reg": "covariance",
                   "pixel_labels_per_step": w.pixel_labels},
        "roofline": roof, "cpu_baseline": cpu, "error": err, "stages": stage_rows,
        "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
