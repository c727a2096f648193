"""Seeded synthetic workloads for the multi-label cost-volume filter.

This module only draws inputs: a colour guidance image made of Voronoi
regions and a truncated-absolute-difference cost volume over a per-region
disparity map.  It contains none of the filter's arithmetic, so the FP64
oracle and the HIP path can both be fed from it without sharing any code
that computes the method.

The structure mirrors the multi-label setting of the paper (Sec. 1: a cost
volume V(x, y, l) whose slices are aggregated by a guided filter before a
winner-takes-all label choice): piecewise-constant colour regions carry
region-wise disparities, which is the structure of a stereo cost volume.

Layouts returned:
  guide  float32 [m][H][W]   (planar channels, values in about [0, 1], not clamped)
  cost   float32 [H][W][L]   (pixel-major, label-contiguous)
  disp   float64 [H][W]      (the disparity the costs were built from)

Random draws, in this order, from ``numpy.random.default_rng(seed)``:
  1. K Voronoi seeds, uniform over [0, W) x [0, H)
  2. K region colours, uniform [0, 1]^m
  3. the disparity model's per-region parameters
  4. guidance noise N(0, sigma_g^2) per pixel and channel
  5. cost noise N(0, sigma_c^2) per pixel and label
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "make_workload",
    "make_workload_device",
    "make_batch_specs",
    "make_request_specs",
    "round_cost",
    "voronoi_regions",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic filtering problem (sizes plus filter parameters)."""

    name: str
    height: int
    width: int
    regions: int
    labels: int
    radius: int
    eps: float
    degree: int
    disparity: str            # "region_int" | "smooth_region" | "planar"
    seed: int
    guide_channels: int = 3
    basis: str = "monomial"   # "monomial" | "power"
    sigma_guide: float = 0.02
    sigma_cost: float = 0.01
    cost_dtype: str = "f32"   # "f32" | "bf16" | "f16"

    @property
    def pixels(self) -> int:
        return self.height * self.width

    @property
    def pixel_labels(self) -> int:
        return self.height * self.width * self.labels

    @property
    def n(self) -> int:
        m, d = self.guide_channels, self.degree
        if self.basis == "power":
            return m * d
        return math.comb(m + d, d) - 1


# Named workloads.  Sizes follow the statement of the problem: a small colour
# case the oracle finishes in seconds, a degree-2 colour case, and a degree-3
# colour case on a wide stereo-sized frame.
WORKLOADS = {
    "rgb64_n3_L16": Workload(
        name="rgb64_n3_L16", height=64, width=64, regions=12, labels=16,
        radius=4, eps=1e-4, degree=1, disparity="region_int", seed=1),
    "voronoi450x375_n9_L60": Workload(
        name="voronoi450x375_n9_L60", height=375, width=450, regions=40,
        labels=60, radius=9, eps=1e-4, degree=2, disparity="smooth_region",
        seed=2),
    "voronoi1242x375_n19_L128": Workload(
        name="voronoi1242x375_n19_L128", height=375, width=1242, regions=80,
        labels=128, radius=9, eps=1e-3, degree=3, disparity="planar", seed=3),
    "voronoi1242x375_n19_L128_bf16": Workload(
        name="voronoi1242x375_n19_L128_bf16", height=375, width=1242,
        regions=80, labels=128, radius=9, eps=1e-3, degree=3,
        disparity="planar", seed=3, cost_dtype="bf16"),
    "voronoi1242x375_n19_L128_f16": Workload(
        name="voronoi1242x375_n19_L128_f16", height=375, width=1242,
        regions=80, labels=128, radius=9, eps=1e-3, degree=3,
        disparity="planar", seed=3, cost_dtype="f16"),
}


def voronoi_regions(seeds_xy: np.ndarray, height: int, width: int) -> np.ndarray:
    """Nearest-seed region index for every pixel centre (x + 0.5, y + 0.5).

    Euclidean distance; ties go to the lower seed index (``argmin`` keeps the
    first minimum).  Rows are processed in chunks to bound memory.
    """
    k = seeds_xy.shape[0]
    out = np.empty((height, width), dtype=np.int32)
    xc = np.arange(width, dtype=np.float64) + 0.5
    rows_per_chunk = max(1, int(4_000_000 // max(1, width * k)))
    for y0 in range(0, height, rows_per_chunk):
        y1 = min(height, y0 + rows_per_chunk)
        yc = np.arange(y0, y1, dtype=np.float64)[:, None] + 0.5
        dx = xc[None, :, None] - seeds_xy[None, None, :, 0]
        dy = yc[:, :, None] - seeds_xy[None, None, :, 1]
        out[y0:y1] = np.argmin(dx * dx + dy * dy, axis=2)
    return out


def _disparity(rng: np.random.Generator, w: Workload, region: np.ndarray,
               seeds_xy: np.ndarray) -> np.ndarray:
    k, L = w.regions, w.labels
    yy, xx = np.meshgrid(np.arange(w.height, dtype=np.float64),
                         np.arange(w.width, dtype=np.float64), indexing="ij")
    if w.disparity == "region_int":
        dk = rng.integers(0, min(L, 16), size=k).astype(np.float64)
        return dk[region]
    if w.disparity == "smooth_region":
        lo, hi = 4.0 * L / 60.0, 55.0 * L / 60.0
        dk = rng.uniform(lo, hi, size=k)
        d = dk[region] + 4.0 * np.sin(2 * np.pi * xx / w.width) * np.cos(
            2 * np.pi * yy / w.height)
        return np.clip(d, 0.0, L - 1.0)
    if w.disparity == "planar":
        s = L / 128.0
        ak = rng.uniform(8.0 * s, 119.0 * s, size=k)
        bk = rng.uniform(-0.05, 0.05, size=k) * s
        ck = rng.uniform(-0.05, 0.05, size=k) * s
        xk = seeds_xy[:, 0][region]
        yk = seeds_xy[:, 1][region]
        d = ak[region] + bk[region] * (xx - xk) + ck[region] * (yy - yk)
        return np.clip(d, 0.0, L - 1.0)
    raise ValueError(f"unknown disparity model {w.disparity!r}")


def _round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), kept as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def round_cost(cost: np.ndarray, cost_dtype: str) -> np.ndarray:
    """Float32 costs rounded to the values of ``cost_dtype`` (round to nearest
    even), kept as float32."""
    if cost_dtype == "bf16":
        return _round_bf16(cost)
    if cost_dtype == "f16":
        return np.ascontiguousarray(cost, dtype=np.float32).astype(np.float16).astype(np.float32)
    return cost


def make_workload(w: Workload, *, with_disparity: bool = False,
                  labels_override: Optional[int] = None):
    """Draw the guide image and cost volume of workload ``w``.

    Returns ``(guide, cost)`` or ``(guide, cost, disp)``.  For ``bf16`` and
    ``f16`` cost workloads the returned float32 cost is already rounded to
    the values of that type (round to nearest even), so the oracle and the
    GPU see the same numbers; the same workload with ``cost_dtype="f32"``
    gives the unrounded costs.
    """
    if labels_override is not None:
        w = dataclasses.replace(w, labels=labels_override)
    rng = np.random.default_rng(w.seed)
    seeds_xy = np.stack([rng.uniform(0, w.width, size=w.regions),
                         rng.uniform(0, w.height, size=w.regions)], axis=1)
    colours = rng.uniform(0.0, 1.0, size=(w.regions, w.guide_channels))
    region = voronoi_regions(seeds_xy, w.height, w.width)
    disp = _disparity(rng, w, region, seeds_xy)
    guide = colours[region].transpose(2, 0, 1) + rng.normal(
        0.0, w.sigma_guide, size=(w.guide_channels, w.height, w.width))
    guide = np.ascontiguousarray(guide, dtype=np.float32)
    cost = np.empty((w.height, w.width, w.labels), dtype=np.float32)
    lab = np.arange(w.labels, dtype=np.float64)
    rows = max(1, int(2_000_000 // max(1, w.width * w.labels)))
    for y0 in range(0, w.height, rows):
        y1 = min(w.height, y0 + rows)
        base = np.minimum(np.abs(lab[None, None, :] - disp[y0:y1, :, None]) / 16.0, 0.5)
        noise = rng.normal(0.0, w.sigma_cost, size=base.shape)
        cost[y0:y1] = (base + noise).astype(np.float32)
    cost = round_cost(cost, w.cost_dtype)
    if with_disparity:
        return guide, cost, disp
    return guide, cost


def make_workload_device(w: Workload, device):
    """Draw workload ``w`` with torch on ``device`` (same recipe, another generator).

    For benchmark sizes whose host generation would take longer than the
    measurement (a 64-image batch holds billions of costs).  The draws follow
    the order and distributions of ``make_workload`` but come from a
    ``torch.Generator`` seeded with ``w.seed``, so the values differ from the
    host generator's.  Returns ``(guide, cost)`` as device tensors: guide
    float32 [m][H][W], cost [H][W][L] float32, or bfloat16 / float16 (round
    to nearest even) for ``bf16`` / ``f16`` workloads.
    """
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(w.seed)
    f64 = dict(dtype=torch.float64, device=device)
    H, W_, K, L, m = w.height, w.width, w.regions, w.labels, w.guide_channels
    sx = torch.rand(K, generator=gen, **f64) * W_
    sy = torch.rand(K, generator=gen, **f64) * H
    colours = torch.rand(K, m, generator=gen, **f64)
    xc = torch.arange(W_, **f64) + 0.5
    region = torch.empty(H, W_, dtype=torch.int64, device=device)
    rows = max(1, (1 << 24) // max(1, W_ * K))
    for y0 in range(0, H, rows):
        y1 = min(H, y0 + rows)
        yc = torch.arange(y0, y1, **f64)[:, None, None] + 0.5
        d2 = (xc[None, :, None] - sx) ** 2 + (yc - sy) ** 2
        region[y0:y1] = torch.argmin(d2, dim=2)  # first minimum on ties
    yy = torch.arange(H, **f64)[:, None].expand(H, W_)
    xx = torch.arange(W_, **f64)[None, :].expand(H, W_)
    if w.disparity == "region_int":
        dk = torch.randint(0, min(L, 16), (K,), generator=gen, device=device).double()
        disp = dk[region]
    elif w.disparity == "smooth_region":
        lo, hi = 4.0 * L / 60.0, 55.0 * L / 60.0
        dk = lo + (hi - lo) * torch.rand(K, generator=gen, **f64)
        disp = (dk[region] + 4.0 * torch.sin(2 * math.pi * xx / W_)
                * torch.cos(2 * math.pi * yy / H)).clamp(0.0, L - 1.0)
    elif w.disparity == "planar":
        s = L / 128.0
        ak = (8.0 + 111.0 * torch.rand(K, generator=gen, **f64)) * s
        bk = (-0.05 + 0.1 * torch.rand(K, generator=gen, **f64)) * s
        ck = (-0.05 + 0.1 * torch.rand(K, generator=gen, **f64)) * s
        disp = (ak[region] + bk[region] * (xx - sx[region]) + ck[region] * (yy - sy[region])
                ).clamp(0.0, L - 1.0)
    else:
        raise ValueError(f"unknown disparity model {w.disparity!r}")
    guide = colours[region].permute(2, 0, 1) + w.sigma_guide * torch.randn(
        m, H, W_, generator=gen, **f64)
    guide = guide.float().contiguous()
    cdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[w.cost_dtype]
    cost = torch.empty(H, W_, L, dtype=cdt, device=device)
    lab = torch.arange(L, dtype=torch.float32, device=device)
    rows = max(1, (1 << 26) // max(1, W_ * L))
    for y0 in range(0, H, rows):
        y1 = min(H, y0 + rows)
        base = ((lab - disp[y0:y1, :, None].float()).abs() / 16.0).clamp(max=0.5)
        noise = torch.randn(y1 - y0, W_, L, generator=gen, dtype=torch.float32, device=device)
        cost[y0:y1] = (base + w.sigma_cost * noise).to(cdt)
    return guide, cost


def make_batch_specs(count: int = 64, seed: int = 4, *, max_width: int = 1920,
                     max_height: int = 1080, min_width: int = 256,
                     min_height: int = 256):
    """Workloads of a mixed batch: uneven sizes, n in {3, 9, 19}, L in {16, 64, 256}, r in {4, 9}.

    Image i is drawn from ``default_rng(1000 * seed + i)``.  The parameter
    draws come from ``default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        width = int(rng.integers(min_width, max_width + 1))
        height = int(rng.integers(min_height, max_height + 1))
        degree = int(rng.choice([1, 2, 3]))
        labels = int(rng.choice([16, 64, 256]))
        radius = int(rng.choice([4, 9]))
        eps = 1e-3 if degree == 3 else 1e-4
        specs.append(Workload(
            name=f"batch{seed}_img{i}", height=height, width=width, regions=40,
            labels=labels, radius=radius, eps=eps, degree=degree,
            disparity="planar", seed=1000 * seed + i))
    return specs


def make_request_specs(count: int, seed: int = 5, *, rate_per_s: float = 200.0,
                       max_width: int = 1920, max_height: int = 1080,
                       min_width: int = 320, min_height: int = 240,
                       min_labels: int = 32, max_labels: int = 256):
    """Requests of an open-loop Poisson stream: arrival time (s) and workload.

    Sizes uniform in [min, max], n in {9, 19}, L uniform in [min_labels,
    max_labels], cost dtype f32 or bf16 with equal odds.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(count):
        width = int(rng.integers(min_width, max_width + 1))
        height = int(rng.integers(min_height, max_height + 1))
        degree = int(rng.choice([2, 3]))
        labels = int(rng.integers(min_labels, max_labels + 1))
        dtype = "bf16" if rng.uniform() < 0.5 else "f32"
        eps = 1e-3 if degree == 3 else 1e-4
        reqs.append((float(arrivals[k]), Workload(
            name=f"req{seed}_{k}", height=height, width=width, regions=40,
            labels=labels, radius=9, eps=eps, degree=degree,
            disparity="planar", seed=1000 * seed + k, cost_dtype=dtype)))
    return reqs
