"""Whole-image oracle results by tiles, computed in worker processes.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by the tests and
the benchmark's accuracy check, never by the product path.

The filter's output at pixel q depends on the coefficients of the pixels p
within r of q (the aggregation of Eq. 7 / Eq. 11), and those depend on the
guidance and cost within r of p (the window statistics of Sec. 5.1).  So the
output rows [y0, y1) are exactly those of the oracle run on the crop of rows
[y0 - 2r, y1 + 2r), clipped to the image: every window that touches an
output row lies inside that crop and is clipped there exactly as in the whole
image.  The same holds along the columns, so output tiles [y0, y1) x [x0, x1)
come from crops with a 2r halo on every side.  This module only cuts the
image into such tiles, runs the oracle functions of ``hgf_oracle`` on each
crop in a process pool and pastes the output tiles back; it does no
arithmetic of its own.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import hgf_oracle as O


def tile_job(G: np.ndarray, V: np.ndarray, r: int, eps: float, box, *, mode: str = "covariance",
             label_chunk: int | None = None):
    """The work of one output tile box = (y0, y1, x0, x1): its crop of G and V
    with a 2r halo on every side (clipped to the image), for ``run_tile``.
    ``label_chunk`` labels per solve (None: the oracle's own choice)."""
    y0, y1, x0, x1 = box
    H, W = V.shape[:2]
    cy0, cy1 = max(0, y0 - 2 * r), min(H, y1 + 2 * r)
    cx0, cx1 = max(0, x0 - 2 * r), min(W, x1 + 2 * r)
    return (np.asarray(G[:, cy0:cy1, cx0:cx1], dtype=np.float64), np.asarray(V[cy0:cy1, cx0:cx1]),
            r, eps, mode, label_chunk, (y0, y1, x0, x1), (cy0, cx0))


def run_tile(job):
    """((y0, x0), Z of the tile) for a job of ``tile_job``."""
    G, V, r, eps, mode, lc, (y0, y1, x0, x1), (cy, cx) = job
    if mode == "covariance":
        Z = O.filter_covariance(G, V, r, eps, label_chunk=lc)
    elif mode == "ridge":
        Z = O.filter_ridge(G, V, r, eps, label_chunk=lc)
    else:
        raise ValueError(f"unknown mode {mode!r}")
    return (y0, x0), Z[y0 - cy:y1 - cy, x0 - cx:x1 - cx]


def default_workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _splits(size: int, parts: int, r: int):
    parts = max(1, min(parts, size // max(1, 4 * r + 1) or 1))
    step = -(-size // parts)
    return [(a, min(size, a + step)) for a in range(0, size, step)]


def filter_image(G: np.ndarray, V: np.ndarray, r: int, eps: float, *, mode: str = "covariance",
                 tiles: tuple[int, int] | None = None, workers: int = 0,
                 label_chunk: int = 16) -> np.ndarray:
    """Z [H][W][L] float64 of the whole image: the values of
    ``filter_covariance`` / ``filter_ridge`` on the full arrays (up to the
    summation order of the box sums), by output tiles (``tiles`` = rows x
    columns of tiles) with a 2r halo on each side, ``label_chunk`` labels per
    solve of each crop.

    G: guidance [n][H][W] (already synthesized); V: cost [H][W][L].  Workers
    are started with the "spawn" method (no fork of a process that may hold
    a GPU runtime) and only run numpy; call it from an importable module or
    a script (not from stdin).
    """
    G = np.asarray(G, dtype=np.float64)
    n, H, W = G.shape
    if V.shape[:2] != (H, W):
        raise ValueError("cost and guidance sizes differ")
    workers = workers or default_workers()
    if tiles is None:
        # about two tiles per worker, split along the longer side first
        ty = max(1, round((2 * workers * H / W) ** 0.5))
        tiles = (ty, max(1, -(-2 * workers // ty)))
    jobs = [tile_job(G, V, r, eps, (y0, y1, x0, x1), mode=mode, label_chunk=label_chunk)
            for y0, y1 in _splits(H, tiles[0], r) for x0, x1 in _splits(W, tiles[1], r)]
    Z = np.empty((H, W, V.shape[2]), dtype=np.float64)

    def put(res):
        (y0, x0), z = res
        Z[y0:y0 + z.shape[0], x0:x0 + z.shape[1]] = z

    if workers == 1 or len(jobs) == 1:
        for j in jobs:
            put(run_tile(j))
        return Z
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(workers, len(jobs))) as pool:
        for res in pool.imap_unordered(run_tile, jobs):
            put(res)
    return Z
