"""Throughput of the HGF cost-volume filter on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--secondary n19,batch,serve | none] [--no-cpu-baseline]

A step is one pass of the whole hot path over one synthetic cost volume that
is already resident in HBM: guidance synthesis, guidance window statistics,
per-pixel inverse, per-label coefficient box sums and solve, coefficient box
filter and output, winner-takes-all labels (one hgf_filter call).  The
headline workload is the 450 x 375 colour Voronoi image with degree-2
polynomial guidance (n = 9), 60 labels, r = 9, eps = 1e-4.

Prints one JSON line: throughput in Mpixel.labels/s, the per-stage kernel
times measured with HIP events on the filter's stream over the timed
region, the roofline position of the dominant kernel, the error of the
filtered costs against the FP64 oracle at sampled pixels, and the oracle's
own throughput on a bounded sample of the same workload on the host cores.
The line's "secondary" list adds the other forms of the metric:
  n19    the 1242 x 375 degree-3 colour image (n = 19, 128 labels, r = 9), float32
         and bfloat16 costs
  batch  64 images of uneven size (n in {3, 9, 19}, L in {16, 64, 256}, r in
         {4, 9}) filtered by one graph replay, against 64 sequential calls
  serve  an open-loop Poisson stream of requests (n in {9, 19}, 32-256 labels,
         float32 / bfloat16 costs) through the serving queue: p50 / p99
         latency from scheduled arrival to completion, sustained throughput
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1803_00005_amd import synth  # noqa: E402
from paper_1803_00005_amd.build_lib import source_hash  # noqa: E402

METRIC = "filtered Mpixel·labels/s (n=9,19) at stated error vs FP64; HBM GB/s; p99"
UNIT = "Mpixel·labels/s"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
# MI355X's published FP32 vector peak (packed / dual-issue FP32 counted)
FP32_PEAK_TFLOPS = 157.3
# FMA rate of the vector ALU without packed FP32: 256 CU x 4 SIMD x 16 lanes x
# 2 flop x 2.4 GHz; float64 FMAs issue at the same rate on this chip.  The
# kernels are built without packed FP32, so this is the rate they can reach.
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
    esz = 4 if w.cost_dtype == "f32" else 2
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


def method_model(w: synth.Workload):
    """The method's own work per px·label, independent of any kernel design.

    Bytes: the algorithmic minimum that must cross HBM: read the cost, write
    Z, plus per pixel the guidance read (4 m) and the label write (4) spread
    over the L labels.  Flops: the coefficient product a = M c (2 n^2), the
    two separable running-sum box filters of the n + 1 product and
    coefficient channels (8 (n + 1)), the products, covariances, intercept and
    output (7 n), plus the per-pixel guidance statistics and inverse
    (n^3 + 4 n (n + 3) / 2) spread over the labels."""
    n, L, m = w.n, w.labels, w.guide_channels
    e = 4 if w.cost_dtype == "f32" else 2
    return {"bytes": e + 4 + (4 * m + 4) / L,
            "flops": 2 * n * n + 8 * (n + 1) + 7 * n + (n ** 3 + 4 * n * (n + 3) / 2) / L}


def method_roofline(w, name, units, ms_per_launch, staged, traffic, ms_step):
    """Roofline position of the dominant kernel: the method's minimum bytes
    and flops of the units (px·labels) one launch processes, over that
    kernel's mean launch time, against 8 TB/s and 157.3 TFLOP/s.  At minimum
    traffic the method is ALU-bound (its intensity is above the ridge), which
    "binding_roof" names; "frac" is the HBM fraction of the algorithmic bytes.
    The staged bytes (the design's own traffic between its kernels), the
    non-packed vector peak and the measured counter traffic are separate
    fields."""
    mm = method_model(w)
    sec = ms_per_launch * 1e-3
    gbs = units * mm["bytes"] / sec / 1e9
    tfs = units * mm["flops"] / sec / 1e12
    intensity = mm["flops"] / mm["bytes"]
    ridge = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    step_s = ms_step * 1e-3
    return {
        "kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
        "units_per_launch": units, "unit_of_work": "px·label",
        "algorithmic_bytes_per_unit": mm["bytes"], "algorithmic_flops_per_unit": mm["flops"],
        "ms_per_launch": ms_per_launch,
        "alu": {"achieved": tfs, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tfs / FP32_PEAK_TFLOPS,
                "frac_of_nonpacked_peak": tfs / VALU_PEAK_TFLOPS,
                "nonpacked_peak": VALU_PEAK_TFLOPS},
        "binding_roof": "alu" if intensity > ridge else "hbm",
        "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
        "whole_step": {"hbm_frac": units * mm["bytes"] / step_s / 1e9 / HBM_PEAK_GBS,
                       "alu_frac": units * mm["flops"] / step_s / 1e12 / FP32_PEAK_TFLOPS},
        "staged": staged,
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


def profile_name(w: synth.Workload, stats: str = "f32") -> str:
    """Name of a workload's profile summaries (the float64 solve has its own)."""
    return w.name + ("_f64" if stats == "f64" else "")


def measured_traffic(workload: str, stage: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current sources of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    name = KERNEL_NAMES.get(stage, "")
    k = rec.get("kernels", {}).get(name, None)
    if not k or k.get("source_hash") != source_hash(name):
        return None
    return k.get("hbm_bytes_per_launch")


# ----------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample, on the host cores
# ----------------------------------------------------------------------------

def _oracle_band(job):
    from threadpoolctl import threadpool_limits

    from oracle import banded
    with threadpool_limits(1):
        t0 = time.perf_counter()
        banded.run_tile(job)
        return time.perf_counter() - t0


def cpu_baseline(w: synth.Workload, guide, cost, target_s: float = 12.0, tile: int = 128):
    """The FP64 oracle on the host cores, on a bounded sample of the workload:
    output tiles of up to ``tile`` x ``tile`` pixels of the real image, each
    computed exactly from its crop with a 2r halo on every side (the halo's
    work counts against the oracle; only the tile's own px·labels count as
    output)."""
    import multiprocessing as mp

    from oracle import banded
    from oracle import hgf_oracle as O
    cores = len(os.sched_getaffinity(0))
    G = O.guidance(guide, w.degree, w.basis)
    boxes = [(y0, min(w.height, y0 + tile), x0, min(w.width, x0 + tile))
             for y0 in range(0, w.height, tile) for x0 in range(0, w.width, tile)]
    # interior tiles first (a full-size tile with a full halo), then the rest
    boxes.sort(key=lambda b: -((b[1] - b[0]) * (b[3] - b[2])))
    job = lambda b: banded.tile_job(G, cost, w.radius, w.eps, b)
    # calibrate on one tile, then size the sample so that every core works ~target_s
    t1 = _oracle_band(job(boxes[0]))
    ntiles = cores * max(1, int(target_s / max(t1, 1e-3)))
    sample = [boxes[k % len(boxes)] for k in range(ntiles)]
    ctx = mp.get_context("fork")   # before anything touches the GPU
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_band, [job(b) for b in sample], chunksize=1)
    wall = time.perf_counter() - t0
    pl = sum((b[1] - b[0]) * (b[3] - b[2]) for b in sample) * w.labels
    a = boxes[0]
    return {"value": pl / wall / 1e6, "unit": UNIT, "cores": cores, "kind": "oracle",
            "workload": w.name,
            "sample": f"{ntiles} output tiles (up to {tile}x{tile} px) x {w.labels} labels of the "
                      f"{w.name} image, each computed exactly from its crop with a "
                      f"{2 * w.radius}-pixel halo (FP64 numpy, per-pixel LU), {cores} processes, "
                      f"{wall:.1f} s wall; one tile on one core: {t1:.2f} s",
            "single_core_value": (a[1] - a[0]) * (a[3] - a[2]) * w.labels / t1 / 1e6}


# ----------------------------------------------------------------------------
# accuracy at sampled pixels against the oracle
# ----------------------------------------------------------------------------

class _DeviceCrop:
    """Host view of a device [H][W][L] tensor that copies only the slices taken."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, idx):
        return self.t[idx].float().cpu().numpy()


def sampled_error(w: synth.Workload, guide, cost, Z, lab, k: int = 14, seed: int = 0):
    """Max error of Z (device) against the FP64 oracle at k random pixels and two corners.

    guide and cost are numpy arrays or device tensors (cost is then read one
    crop at a time)."""
    from oracle import hgf_oracle as O
    g = guide if isinstance(guide, np.ndarray) else guide.cpu().numpy()
    v = cost if isinstance(cost, np.ndarray) else _DeviceCrop(cost)
    rng = np.random.default_rng(seed)
    pts = sorted({(0, 0), (w.height - 1, w.width - 1)} |
                 {(int(rng.integers(0, w.height)), int(rng.integers(0, w.width)))
                  for _ in range(k)})
    idx = tuple(np.array(pts).T)
    Zo = O.filter_points(O.guidance(g, w.degree, w.basis), v, w.radius, w.eps, pts)
    vmax = max(float(np.abs(v[y, x]).max()) for (y, x) in pts)
    if isinstance(cost, np.ndarray):
        vmax = float(np.abs(cost).max())
    scale = np.maximum(np.abs(Zo), vmax)
    Zg = Z[idx].double().cpu().numpy() if not isinstance(Z, np.ndarray) else Z[idx]
    lg = lab[idx].cpu().numpy() if not isinstance(lab, np.ndarray) else lab[idx]
    rel = float(np.max(np.abs(Zg - Zo) / scale))
    agree = bool(np.all((lg == O.wta(Zo)) | O.near_tie_mask(Zo)))
    return {"max_rel_vs_fp64_oracle": rel, "tolerance": 1e-4, "points": len(pts),
            "labels_agree_outside_near_ties": agree}


# ----------------------------------------------------------------------------
# plain form: one image per call
# ----------------------------------------------------------------------------

def run_plain(ctx, w, g_d, c_d, steps, warmup, stage_timing=True, autotune=True, stats="f32"):
    import torch

    from paper_1803_00005_amd import hgf
    dev = g_d.device
    p = hgf.make_params(w.height, w.width, w.labels, radius=w.radius, eps=w.eps, degree=w.degree,
                        guide_channels=w.guide_channels, basis=w.basis, cost_dtype=w.cost_dtype,
                        stats_dtype=stats)
    ws = torch.empty(hgf.workspace_size(p), dtype=torch.uint8, device=dev)
    Z = torch.empty((w.height, w.width, w.labels), dtype=torch.float32, device=dev)
    lab = torch.empty((w.height, w.width), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        ctx.filter(g_d, c_d, radius=w.radius, eps=w.eps, degree=w.degree, basis=w.basis,
                   stats_dtype=stats, out=Z, labels=lab, workspace=ws, stream=stream)

    if autotune:
        # untimed set-up: the strip decomposition for this size class is chosen
        # by timing the candidates on these inputs (hgf_autotune)
        ctx.autotune(g_d, c_d, radius=w.radius, eps=w.eps, degree=w.degree, basis=w.basis,
                     stats_dtype=stats, stream=stream)
    mode = 1 if stats == "f64" else 0   # the solve form column of the tuning table
    tuned = [r for r in ctx.tune_entries() if r[1] == w.n and r[2] == w.radius and r[3] == mode
             and r[4] == hgf.COST_DTYPES[w.cost_dtype]
             and r[5] == (w.pixels.bit_length() - 1)]
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed():
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the headline: the plain calls, no instrumentation
    ms = timed()
    # the same steps again with an event pair around every kernel stage on the
    # launch stream: per-kernel launch durations for the roofline (the events
    # themselves cost about 0.1 ms per step, so this pass is not the headline)
    stages, ms_staged = {}, None
    if stage_timing:
        ctx.set_stage_timing(True)
        ctx.stage_times()
        ms_staged = timed()
        stages = ctx.stage_times()
        ctx.set_stage_timing(False)

    model = stage_model(w)
    rows = []
    for name in STAGES:
        if name not in stages or stages[name][1] == 0:
            continue
        tot, cnt = stages[name]
        per = tot / cnt
        mdl = {k: v / (cnt / steps) for k, v in model[name].items()}
        rf = roofline_of(name, mdl, per, None)
        rows.append({"stage": name, "ms_per_step": tot / steps, "launches": cnt,
                     "ms_per_launch": per, "bound": rf["bound"],
                     "achieved": round(rf["achieved"], 3), "unit": rf["unit"],
                     "frac": round(rf["frac"], 4)})
    roof = None
    if rows:
        dom = max(rows, key=lambda r: r["ms_per_step"])
        cnt = stages[dom["stage"]][1]
        per_step = cnt / steps
        mdl = {k: v / per_step for k, v in model[dom["stage"]].items()}
        st = roofline_of(KERNEL_NAMES.get(dom["stage"], dom["stage"]), mdl,
                         dom["ms_per_launch"], None)
        staged = {"bytes_per_launch": mdl["bytes"], "flops_per_launch": mdl["flops"],
                  "bound": st["bound"], "achieved": st["achieved"], "unit": st["unit"],
                  "peak": st["peak"], "frac": st["frac"]}
        roof = method_roofline(w, KERNEL_NAMES.get(dom["stage"], dom["stage"]),
                               w.pixel_labels / per_step, dom["ms_per_launch"], staged,
                               measured_traffic(profile_name(w, stats), dom["stage"]), ms)
    return {"ms": ms, "ms_stage_timed": ms_staged, "stages": rows, "roofline": roof, "Z": Z,
            "labels": lab,
            "tuning": {["coef", "out", "moments"][r[0]]: r[6] for r in tuned}}


def secondary_c1(ctx, reps=2000):
    """The 64 x 64 colour workload (n = 3, 16 labels), which is launch-bound:
    the latency of one filter call, back to back and alone (synchronised
    after each call), and of the allocation-free call captured once in a
    graph and replayed."""
    import torch
    w = synth.WORKLOADS["rgb64_n3_L16"]
    guide, cost = synth.make_workload(w)
    g = torch.from_numpy(guide).cuda()
    c = torch.from_numpy(cost).cuda()
    Z = torch.empty((w.height, w.width, w.labels), dtype=torch.float32, device="cuda")
    lab = torch.empty((w.height, w.width), dtype=torch.int32, device="cuda")
    from paper_1803_00005_amd import hgf
    ws = torch.empty(hgf.workspace_size(hgf.make_params(
        w.height, w.width, w.labels, radius=w.radius, eps=w.eps, degree=w.degree)),
        dtype=torch.uint8, device="cuda")
    f = lambda: ctx.filter(g, c, radius=w.radius, eps=w.eps, degree=w.degree, out=Z, labels=lab,
                           workspace=ws)
    for _ in range(20):
        f()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        f()
    e1.record()
    torch.cuda.synchronize()
    back_to_back = e0.elapsed_time(e1) / reps
    t0 = time.perf_counter()
    for _ in range(200):
        f()
        torch.cuda.synchronize()
    alone = (time.perf_counter() - t0) / 200 * 1e3
    rec = {"form": "latency", "workload": w.name, "pixel_labels": w.pixel_labels,
           "ms_per_call_back_to_back": back_to_back, "ms_per_call_synchronised": alone,
           "value": w.pixel_labels / back_to_back / 1e3, "unit": UNIT}
    Zref, lref = Z.clone(), lab.clone()
    try:
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ctx.filter_static(g, c, Z, lab, radius=w.radius, eps=w.eps, degree=w.degree)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=st):
            ctx.filter_static(g, c, Z, lab, radius=w.radius, eps=w.eps, degree=w.degree)
        same = True
        for _ in range(3):   # replays with eager work and synchronisation between them
            Z.zero_()
            graph.replay()
            torch.cuda.synchronize()
            same = same and torch.equal(Z, Zref) and torch.equal(lab, lref)
        e0.record()
        for _ in range(reps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        rec["ms_per_graph_replay"] = e0.elapsed_time(e1) / reps
        rec["graph_equals_eager_bitwise"] = bool(same)
    except Exception as e:  # the plain-call figures stand on their own
        rec["graph_error"] = repr(e)[:200]
    say(f"c1 latency: {back_to_back * 1e3:.1f} us back to back, {alone * 1e3:.1f} us alone, "
        f"graph {rec.get('ms_per_graph_replay', float('nan')) * 1e3:.1f} us")
    return rec


N19_FORMS = [("voronoi1242x375_n19_L128", "f32"), ("voronoi1242x375_n19_L128", "f64"),
             ("voronoi1242x375_n19_L128_bf16", "f64"), ("voronoi1242x375_n19_L128_f16", "f64")]


def secondary_n19(ctx, steps, warmup, check, autotune=True):
    """The degree-3 workload: float32 costs with the float32 and the float64
    solve, and the precision forms (bfloat16 / float16 costs, float64 solve)."""
    import torch
    out = []
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    for name, stats in N19_FORMS:
        w = synth.WORKLOADS[name]
        say(f"n19: {name}, {stats} solve")
        guide, cost = synth.make_workload(w)
        g_d = torch.from_numpy(guide).cuda()
        c_d = torch.from_numpy(cost).cuda().to(tdt[w.cost_dtype])
        r = run_plain(ctx, w, g_d, c_d, steps, warmup, autotune=autotune, stats=stats)
        rec = {"form": "plain", "workload": w.name, "value": w.pixel_labels / r["ms"] / 1e3,
               "tuning": {"target_blocks": r["tuning"]},
               "unit": UNIT, "ms_per_step": r["ms"], "n": w.n, "labels": w.labels,
               "cost_dtype": w.cost_dtype, "stats_dtype": stats, "roofline": r["roofline"],
               "stages": r["stages"], "ms_per_step_stage_timed": r["ms_stage_timed"]}
        if check:
            rec["error"] = sampled_error(w, guide, cost, r["Z"], r["labels"])
        out.append(rec)
        say(f"n19: {name} {stats} {r['ms']:.3f} ms/step")
        del g_d, c_d, r
        torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------------------
# batched form: one graph replay over 64 images of uneven size
# ----------------------------------------------------------------------------

def secondary_batch(ctx, count, steps, warmup, check):
    import torch

    from paper_1803_00005_amd import hgf
    dev = torch.device("cuda", 0)
    specs = synth.make_batch_specs(count, seed=4)
    say(f"batch: drawing {count} images on the device")
    data = [synth.make_workload_device(w, dev) for w in specs]
    outs = [(torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev),
             torch.empty(w.height, w.width, dtype=torch.int32, device=dev)) for w in specs]
    items = [dict(guide=g, cost=c, radius=w.radius, eps=w.eps, degree=w.degree)
             for w, (g, c) in zip(specs, data)]
    total = sum(w.pixel_labels for w in specs)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(max(1, warmup)):
        ctx.filter_batch(items, outputs=outs, stream=stream)  # first call captures the graph
    torch.cuda.synchronize()
    say("batch: graph captured")
    e0.record(stream)
    for _ in range(steps):
        ctx.filter_batch(items, outputs=outs, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / steps
    say(f"batch: {ms_graph:.2f} ms per replay")
    # the same images one hgf_filter call after another on the same stream
    wsz = max(hgf.workspace_size(hgf.make_params(w.height, w.width, w.labels, radius=w.radius,
                                                 eps=w.eps, degree=w.degree,
                                                 cost_dtype=w.cost_dtype)) for w in specs)
    ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    seq_out = [(torch.empty_like(z), torch.empty_like(lb)) for z, lb in outs[:4]]

    def sequential(check_first=False):
        for i, (w, (g, c)) in enumerate(zip(specs, data)):
            z, lb = seq_out[i] if check_first and i < 4 else outs[i]
            ctx.filter(g, c, radius=w.radius, eps=w.eps, degree=w.degree, out=z, labels=lb,
                       workspace=ws, stream=stream)

    sequential(check_first=True)
    torch.cuda.synchronize()
    equal = all(torch.equal(outs[i][0], seq_out[i][0]) and torch.equal(outs[i][1], seq_out[i][1])
                for i in range(min(4, count)))
    e0.record(stream)
    sequential()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1)
    say(f"batch: sequential {ms_seq:.2f} ms")
    rec = {"form": "batch", "workload": f"batch{count}_mixed", "images": count,
           "value": total / ms_graph / 1e3, "unit": UNIT, "ms_per_step": ms_graph,
           "pixel_labels_per_step": total, "sequential_ms": ms_seq,
           "speedup_vs_sequential": ms_seq / ms_graph,
           "graph_equals_sequential_bitwise_first4": bool(equal),
           "data": "device-drawn (torch generator), same recipe"}
    if check:
        # the two smallest images, and the image with the most coefficient
        # workspace (the one most likely to run several launch groups)
        order = sorted(range(count), key=lambda i: specs[i].pixels)[:2]
        big = max(range(count), key=lambda i: specs[i].pixel_labels * (specs[i].n + 1))
        order.append(big)
        groups = {}
        for i in order:
            w_ = specs[i]
            per_chunk = w_.pixels * (w_.n + 1) * 64 * 4
            groups[i] = -(-((w_.labels + 63) // 64) // max(1, (12 << 30) // per_chunk))
        rec["error"] = [dict(image=i, launch_groups=groups[i],
                             **sampled_error(specs[i], data[i][0], data[i][1], outs[i][0],
                                             outs[i][1], k=4))
                        for i in order]
    del data, outs, seq_out, ws
    torch.cuda.empty_cache()
    return rec


# ----------------------------------------------------------------------------
# serving form: open-loop Poisson arrivals through the serving queue
# ----------------------------------------------------------------------------

class _ServePool:
    """Device inputs and outputs of the served streams: ``size`` distinct
    requests drawn from the serving mix (sizes, labels, n, cost dtype), each
    with its own Voronoi inputs; request k of a stream uses entry k mod size."""

    def __init__(self, size, seed=5):
        import torch
        dev = torch.device("cuda", 0)
        self.specs = [w for _, w in synth.make_request_specs(size, seed=seed)]
        self.inputs = [synth.make_workload_device(w, dev) for w in self.specs]
        self.outputs = [(torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev),
                         torch.empty(w.height, w.width, dtype=torch.int32, device=dev))
                        for w in self.specs]


def _serve_stream(ctx, pool, requests, rate, slots, arena_gb, seed):
    """One open-loop Poisson stream through the serving queue.  Latency is
    measured from each request's scheduled arrival to its completion on the
    device clock (queueing, admission and any wait for a free input buffer
    included)."""
    import torch

    from paper_1803_00005_amd import hgf
    npool = len(pool.specs)
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    srv = hgf.Server(ctx, slots=slots, arena_bytes=int(arena_gb * (1 << 30)),
                     max_queue=requests + 1)
    # warm-up: every pool entry once, alone (code objects, caches)
    for j in range(npool):
        w = pool.specs[j]
        srv.submit(pool.inputs[j][0], pool.inputs[j][1], pool.outputs[j][0], pool.outputs[j][1],
                   radius=w.radius, eps=w.eps, degree=w.degree)
        srv.drain()
    srv.poll(4 * npool)
    torch.cuda.synchronize()
    dev0 = srv.now_ms()
    t0 = time.perf_counter()
    done, id_of = {}, {}
    last_note = t0

    def collect():
        for c in srv.poll(1024):
            done[c.id] = c

    k = 0
    while k < requests:
        now = time.perf_counter() - t0
        if time.perf_counter() - last_note > 10.0:
            say(f"serve: {k} of {requests} submitted, {len(done)} done")
            last_note = time.perf_counter()
        if now < arrivals[k]:
            collect()
            if arrivals[k] - now > 5e-4:
                time.sleep(2e-4)
            continue
        j = k % npool
        if k >= npool:  # request k writes the buffers of request k - npool
            while id_of[k - npool] not in done:
                collect()
        w = pool.specs[j]
        id_of[k] = srv.submit(pool.inputs[j][0], pool.inputs[j][1], pool.outputs[j][0],
                              pool.outputs[j][1], radius=w.radius, eps=w.eps, degree=w.degree)
        k += 1
    srv.drain()
    collect()
    stats = srv.stats()
    srv.close()
    lat = np.array([done[id_of[k]].end_ms - (dev0 + 1e3 * arrivals[k]) for k in range(requests)])
    statuses = sorted({int(done[id_of[k]].status) for k in range(requests)})
    work = np.array([pool.specs[k % npool].pixel_labels for k in range(requests)],
                    dtype=np.float64)
    span_ms = max(done[id_of[k]].end_ms for k in range(requests)) - dev0
    offered = work.sum() / max(arrivals[-1], 1e-9) / 1e6
    value = work.sum() / span_ms / 1e3
    return {"rate_per_s": rate, "requests": requests, "value": value, "unit": UNIT,
            "offered": offered, "sustained": bool(value >= 0.95 * offered),
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "max": float(lat.max()),
                           "first_half_p99": float(np.percentile(lat[:requests // 2], 99)),
                           "second_half_p99": float(np.percentile(lat[requests // 2:], 99))},
            "span_s": span_ms / 1e3, "arrival_span_s": float(arrivals[-1]),
            "arena_peak_gb": stats["arena_peak"] / (1 << 30), "statuses": statuses,
            "mean_pixel_labels_per_request": float(work.mean())}


def secondary_serve(ctx, requests, pool_size, rate, slots, arena_gb, low_rate, low_requests):
    """The serving form: the Poisson stream of the serving workload (its rate
    and request count), and a second stream below the device's capacity so
    that a steady-state p50 / p99 is measured too.  Served results are
    checked bit for bit against hgf_filter alone."""
    import torch
    say(f"serve: drawing {pool_size} distinct requests on the device")
    pool = _ServePool(pool_size)
    say(f"serve: stream of {requests} requests at {rate} req/s")
    main = _serve_stream(ctx, pool, requests, rate, slots, arena_gb, seed=50)
    say(f"serve: p50 {main['latency_ms']['p50']:.1f} ms p99 {main['latency_ms']['p99']:.1f} ms, "
        f"{main['value']:.0f} of {main['offered']:.0f} {UNIT} offered")
    low = None
    if low_requests > 0:
        say(f"serve: stream of {low_requests} requests at {low_rate} req/s")
        low = _serve_stream(ctx, pool, low_requests, low_rate, slots, arena_gb, seed=51)
        say(f"serve: p50 {low['latency_ms']['p50']:.1f} ms p99 {low['latency_ms']['p99']:.1f} ms "
            f"at {low_rate} req/s")
    # alone vs in the mix: the last use of three pool entries through hgf_filter
    same = True
    for j in range(min(3, pool_size)):
        w = pool.specs[j]
        z, lb = ctx.filter(pool.inputs[j][0], pool.inputs[j][1], radius=w.radius, eps=w.eps,
                           degree=w.degree)
        torch.cuda.synchronize()
        same = same and torch.equal(z, pool.outputs[j][0]) and torch.equal(lb, pool.outputs[j][1])
    # the plain path on the same requests (after the check above, which reads
    # the served outputs): every pool entry once, back to back through
    # hgf_filter on one stream (no queueing, no overlap)
    from paper_1803_00005_amd import hgf
    wsz = max(hgf.workspace_size(hgf.make_params(
        w.height, w.width, w.labels, radius=w.radius, eps=w.eps, degree=w.degree,
        cost_dtype=w.cost_dtype)) for w in pool.specs)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for j, w in enumerate(pool.specs):
        ctx.filter(pool.inputs[j][0], pool.inputs[j][1], radius=w.radius, eps=w.eps,
                   degree=w.degree, out=pool.outputs[j][0], labels=pool.outputs[j][1],
                   workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    plain_value = sum(w.pixel_labels for w in pool.specs) / plain_ms / 1e3
    del ws
    say(f"serve: plain path on the pool {plain_value:.0f} {UNIT}")
    rec = {"form": "serve", "workload": f"poisson{int(rate)}rps_{requests}req",
           "distinct_inputs": pool_size, "slots": slots, "arena_gb": arena_gb,
           **main, "below_capacity": low, "served_equals_alone_bitwise": bool(same),
           "plain_path": {"value": plain_value, "unit": UNIT, "ms": plain_ms,
                          "what": f"the {pool_size} pool requests through hgf_filter back to "
                                  "back on one stream"},
           "data": "device-drawn (torch generator), same recipe; request k of a stream uses the "
                   f"shape and inputs of entry k mod {pool_size} of a pool drawn from the "
                   "serving mix"}
    del pool
    torch.cuda.empty_cache()
    return rec


# ----------------------------------------------------------------------------
# batched SPD inverse (Prop. 1) against the vendor solver's batched inverses
# ----------------------------------------------------------------------------

def secondary_inverse(count=1_000_000, sizes=(3, 5, 7, 9, 11, 13, 15, 17, 19), reps=5):
    import torch

    from paper_1803_00005_amd import hgf
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    rows = []
    for D in sizes:
        gen.manual_seed(100 + D)
        X = torch.rand(count, D + 2, D, generator=gen, dtype=torch.float64, device=dev)
        A = torch.bmm(X.transpose(1, 2).contiguous(), X)
        A += 1e-3 * torch.eye(D, dtype=torch.float64, device=dev)
        del X

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                out = fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps, out

        ms_h, Mh = timed(lambda: hgf.spd_inverse(A))
        ms_lu, Ml = timed(lambda: torch.linalg.inv(A))
        ms_ch, _ = timed(lambda: torch.cholesky_inverse(torch.linalg.cholesky(A)))
        rel = float(((Mh - Ml).abs().amax(dim=(1, 2)) / Ml.abs().amax(dim=(1, 2))).max())
        rows.append({"D": D, "ms_prop1": ms_h, "ms_lu": ms_lu, "ms_cholesky": ms_ch,
                     "matrices_per_s": count / ms_h * 1e3, "speedup_vs_lu": ms_lu / ms_h,
                     "speedup_vs_cholesky": ms_ch / ms_h, "max_rel_vs_lu": rel})
        say(f"inverse D={D}: {ms_h:.3f} ms (LU {ms_lu:.3f}, Cholesky {ms_ch:.3f})")
        del A, Mh, Ml
        torch.cuda.empty_cache()
    return {"form": "spd_inverse", "workload": f"spd{count}_D3-19", "matrices": count,
            "reference": "torch.linalg.inv and torch.cholesky_inverse (vendor batched solver), "
                         "float64", "rows": rows}


# ----------------------------------------------------------------------------
# gray guidance, power basis, one slice: the setting of the paper's timing tables
# ----------------------------------------------------------------------------

# the paper's own GPU times (Table 2, a GTX 960 with ArrayFire): context only
PAPER_TABLE2_MS = {250: {3: 3.9, 5: 10.7, 7: 39.9, 9: 110.2},
                   500: {3: 3.7, 5: 11.1, 7: 40.1, 9: 112.4},
                   1000: {3: 4.1, 5: 10.9, 7: 41.3, 9: 115.9},
                   2000: {3: 4.3, 5: 11.2, 7: 42.7, 9: 121.8}}


def sampled_error_ridge(w: synth.Workload, guide, cost, Z, k: int = 8, seed: int = 0):
    """Max error of a one-label ridge-form Z (device) against the FP64 oracle at k
    random pixels and two corners."""
    from oracle import hgf_oracle as O
    g = guide.cpu().numpy()
    v = _DeviceCrop(cost)
    rng = np.random.default_rng(seed)
    pts = sorted({(0, 0), (w.height - 1, w.width - 1)} |
                 {(int(rng.integers(0, w.height)), int(rng.integers(0, w.width)))
                  for _ in range(k)})
    Zo = O.filter_points(O.guidance(g, w.degree, w.basis), v, w.radius, w.eps, pts, mode="ridge")
    vmax = max(float(np.abs(v[y, x]).max()) for (y, x) in pts)
    idx = tuple(np.array(pts).T)
    Zg = Z[idx].double().cpu().numpy()
    rel = float(np.max(np.abs(Zg - Zo) / np.maximum(np.abs(Zo), vmax)))
    return {"max_rel_vs_fp64_oracle": rel, "tolerance": 1e-4, "points": len(pts)}


def secondary_gray(ctx, sizes=(250, 500, 1000, 2000), ns=(3, 5, 7, 9), reps=10, check=True):
    import torch

    from paper_1803_00005_amd import hgf
    dev = torch.device("cuda", 0)
    rows = []
    for side in sizes:
        for n in ns:
            w = synth.Workload(name=f"gray{side}_n{n}", height=side, width=side, regions=40,
                               labels=1, radius=7, eps=0.05, degree=n, disparity="planar",
                               seed=9000 + side + n, guide_channels=1, basis="power")
            g, c = synth.make_workload_device(w, dev)
            p = hgf.make_params(side, side, 1, radius=w.radius, eps=w.eps, degree=n,
                                guide_channels=1, basis="power", reg="ridge")
            ws = torch.empty(hgf.workspace_size(p), dtype=torch.uint8, device=dev)
            Z = torch.empty((side, side, 1), dtype=torch.float32, device=dev)
            f = lambda: ctx.filter(g, c, radius=w.radius, eps=w.eps, degree=w.degree,
                                   basis="power", reg="ridge", want_labels=False, out=Z,
                                   workspace=ws)
            f()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                f()
            e1.record()
            torch.cuda.synchronize()
            row = {"side": side, "n": n, "ms": e0.elapsed_time(e1) / reps,
                   "paper_gtx960_ms": PAPER_TABLE2_MS[side][n]}
            if check and side == sizes[-1]:
                row["error"] = sampled_error_ridge(w, g, c, Z)
            rows.append(row)
            del g, c, ws, Z
    say("gray sweep: " + ", ".join(f"{r['side']}/{r['n']}: {r['ms']:.3f} ms" for r in rows[-4:]))
    return {"form": "gray_power_ridge", "workload": "gray_power_r7_lambda0.05_L1",
            "note": "one slice (L = 1) per filter, ridge form of Eq. 6 with the power basis; the "
                    "paper's Table 2 times are from other hardware, for context",
            "rows": rows}


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(synth.WORKLOADS))
    ap.add_argument("--stats-dtype", default="f32", choices=("f32", "f64"),
                    help="precision of the per-pixel solve of the timed workload")
    ap.add_argument("--secondary", default="c1,n19,batch,serve,inverse,gray",
                    help="comma list of c1, n19, batch, serve, inverse, gray, or 'none'")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-low-rate", type=float, default=80.0,
                    help="rate of the second, below-capacity stream (req/s)")
    ap.add_argument("--serve-low-requests", type=int, default=1500)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-arena-gb", type=float, default=96.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--tune-file", default=None,
                    help="tuning table to load (default: the one shipped with the package, "
                         "if present); 'none' keeps the built-in defaults")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the strip decomposition on each plain workload before timing it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device fill and sums (reference for the HBM "
                         "byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(across GPUs the filter would shard by label ranges or image strips)",
              file=sys.stderr)
        sys.exit(2)
    secondary = [] if args.secondary == "none" else [x for x in args.secondary.split(",") if x]
    for x in secondary:
        if x not in ("c1", "n19", "batch", "serve", "inverse", "gray"):
            ap.error(f"unknown secondary form {x!r}")

    w = synth.WORKLOADS[args.workload]
    say(f"workload {w.name}: {w.height}x{w.width} n={w.n} L={w.labels} r={w.radius} "
        f"eps={w.eps} cost={w.cost_dtype}")
    guide, cost = synth.make_workload(w)

    # the host-core oracle runs before the GPU is touched (forked workers)
    cpu = cpu_n19 = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, guide, cost)
        say(f"cpu baseline {cpu['value']:.3f} {UNIT} on {cpu['cores']} cores")
        if "n19" in secondary:
            w19 = synth.WORKLOADS["voronoi1242x375_n19_L128"]
            cpu_n19 = cpu_baseline(w19, *synth.make_workload(w19))
            say(f"cpu baseline n19 {cpu_n19['value']:.3f} {UNIT} on {cpu_n19['cores']} cores")

    import torch

    from paper_1803_00005_amd import hgf

    dev = torch.device("cuda", 0)
    g_d = torch.from_numpy(guide).to(dev)
    c_d = torch.from_numpy(cost).to(dev).to(
        {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[w.cost_dtype])
    ctx = hgf.Context(0)
    from paper_1803_00005_amd import tune_table
    tune_file = args.tune_file if args.tune_file is not None else (
        tune_table.DEFAULT_TABLE if os.path.exists(tune_table.DEFAULT_TABLE) else "none")
    if tune_file != "none":
        ctx.tune_load(tune_file)
        say(f"tuning table {tune_file}: {len(ctx.tune_entries())} entries")
    tuning_source = "autotune" if args.autotune else (
        os.path.relpath(tune_file, ROOT) if tune_file != "none" else "built-in defaults")

    if args.copy_calibration:
        # a fill (writes 1 GiB) and a sum (reads 1 GiB): known byte counts for
        # the HBM byte counters
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        for _ in range(3):
            s_ = src.sum()
        torch.cuda.synchronize()
        say(f"copy calibration: fill and 3 sums of {src.numel() * 4} bytes (sum={float(s_):.0f})")
        del src

    t0 = time.perf_counter()
    r = run_plain(ctx, w, g_d, c_d, args.steps, args.warmup, not args.no_stage_timing,
                  autotune=args.autotune, stats=args.stats_dtype)
    ms = r["ms"]
    say(f"timed {args.steps} steps: {ms:.4f} ms/step (wall {time.perf_counter() - t0:.3f} s)")
    value = w.pixel_labels / (ms * 1e-3) / 1e6
    err = None if args.no_check else sampled_error(w, guide, cost, r["Z"], r["labels"])

    sec = []
    if "c1" in secondary:
        sec.append(secondary_c1(ctx))
    if "n19" in secondary:
        sec += secondary_n19(ctx, max(3, args.steps // 2), args.warmup, not args.no_check,
                             autotune=args.autotune)
        if cpu_n19 is not None:
            sec[-len(N19_FORMS)]["cpu_baseline"] = cpu_n19
    if "batch" in secondary:
        sec.append(secondary_batch(ctx, args.batch_count, args.batch_steps, 1,
                                   not args.no_check))
    if "inverse" in secondary:
        sec.append(secondary_inverse())
    if "gray" in secondary:
        sec.append(secondary_gray(ctx, check=not args.no_check))
    if "serve" in secondary:
        sec.append(secondary_serve(ctx, args.serve_requests, args.serve_pool, args.serve_rate,
                                   args.serve_slots, args.serve_arena_gb, args.serve_low_rate,
                                   args.serve_low_requests))

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "height": w.height, "width": w.width, "labels": w.labels,
                   "n": w.n, "degree": w.degree, "basis": w.basis, "radius": w.radius,
                   "eps": w.eps, "cost_dtype": w.cost_dtype, "reg": "covariance",
                   "stats_dtype": args.stats_dtype,
                   "pixel_labels_per_step": w.pixel_labels},
        "roofline": r["roofline"], "cpu_baseline": cpu, "error": err, "stages": r["stages"],
        "ms_per_step_stage_timed": r["ms_stage_timed"],
        "tuning": {"source": tuning_source, "target_blocks": r["tuning"]},
        "secondary": sec, "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
