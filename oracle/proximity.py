"""Proximity loop-closure edges of the patch graph -- test infrastructure.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg use this
module; the product path never imports it.

DPV-SLAM, Sec. 3.2 ("Proximity Loop Closure", "Constructing the Patch
Graph"): loops are detected from the cameras' proximity to previously
visited locations, and long-range edges are inserted from the stored patches
of old frames to recently observed frames.  The edges are uni-directional
(patch of the old frame -> recent frame) because the correlation of eq. 4
only needs the dense features of the destination frame, and with inverse
depths every edge constrains both poses whatever its direction.

Readings where the paper is silent (the same rule defines the global-BA
workload's loop edges):
  * frame i is "old" for frame j when j - i > min_gap; j must be a recent
    frame, j >= first_recent;
  * the pair is a loop when the camera centres (the translations of the
    camera-to-world poses) are closer than `radius`: |c_i - c_j|^2 < r^2;
  * each old frame keeps its max_targets nearest loop frames (ties -> the
    lower frame index), listed in increasing frame order;
  * every patch of the old frame gets one edge to each of them; edges are
    emitted by old frame, then patch, then target frame.
The decisions are integer results of floating-point comparisons, so they
are taken in float32 with a fixed operation order,
d2 = (dx*dx + dy*dy) + dz*dz from float32 centre differences and
r2 = radius*radius rounded to float32, exactly as the device computes them.
"""
from __future__ import annotations

import numpy as np


def squared_distances(centres: np.ndarray, i: int, js: np.ndarray) -> np.ndarray:
    """float32 |c_j - c_i|^2 for the frames js, each operation rounded to float32."""
    c = np.asarray(centres, dtype=np.float32)
    d = c[js] - c[i]
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


def loop_targets(centres, first_recent: int, min_gap: int, radius: float, max_targets: int):
    """Per frame i: the sorted list of its loop target frames."""
    c = np.asarray(centres, dtype=np.float32)
    n = c.shape[0]
    r2 = np.float32(radius) * np.float32(radius)
    out = []
    for i in range(n):
        js = np.arange(max(first_recent, i + min_gap + 1), n)
        if js.size == 0 or max_targets <= 0:
            out.append([])
            continue
        d2 = squared_distances(c, i, js)
        keep = d2 < r2
        cand, dd = js[keep], d2[keep]
        order = np.lexsort((cand, dd))[:max_targets]  # nearest first, ties -> lower j
        out.append(sorted(int(j) for j in cand[order]))
    return out


def loop_edges(targets, patch_off):
    """(ii, jj, kk) int32 of the loop edges: old frame, then patch, then target."""
    ii, jj, kk = [], [], []
    for i, tg in enumerate(targets):
        for k in range(int(patch_off[i]), int(patch_off[i + 1])):
            for j in tg:
                ii.append(i)
                jj.append(j)
                kk.append(k)
    return (np.asarray(ii, dtype=np.int32), np.asarray(jj, dtype=np.int32), np.asarray(kk, dtype=np.int32))
