"""Autotuner of the tile shape (patches per tile) for batched solves.

The tile kernel's cost per edge depends on how many patches share a tile:
more patches amortise the per-tile work (slot poses, the U^T U product) but
produce fewer, longer workgroups and a larger shared-memory footprint.  The
best size depends on the problem's shape, so problems are grouped into size
buckets (patches per frame, edges per patch), and for each bucket a few
member problems are solved as a small batch with every candidate size; the
fastest candidate is kept.  Results are cached in a JSON file keyed by the
bucket, the precision and the device name, so later runs skip the timing.

Everything is timed through the library (HIP events on the solve stream);
this module only chooses arguments.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import binding as B

CANDIDATES = (16, 24, 32, 48, 64, 96, 128)


def bucket_of(n_frames: int, n_patches: int, n_edges: int) -> str:
    """Size bucket of one problem: patches per frame and edges per patch, each
    on a grid of half powers of two (index round(2 log2 x))."""
    ppf = n_patches / max(n_frames, 1)
    epp = n_edges / max(n_patches, 1)
    h = lambda x: int(round(2 * np.log2(max(x, 1.0))))
    return f"ppf{h(ppf)}_epp{h(epp)}"


def _device_name() -> str:
    try:
        return torch.cuda.get_device_name(0)
    except Exception:  # pragma: no cover
        return "unknown"


class TileTuner:
    """Chooses patches-per-tile per size bucket and caches the choices."""

    def __init__(self, cache_path: str | None = None, candidates=CANDIDATES, members: int = 4,
                 steps: int = 5):
        self.cache_path = cache_path
        self.candidates = tuple(candidates)
        self.members = members
        self.steps = steps
        self.table: dict = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = json.load(f)

    def _key(self, bucket: str, precision: int) -> str:
        return f"{_device_name()}|p{precision}|{bucket}"

    def save(self):
        if self.cache_path:
            os.makedirs(os.path.dirname(os.path.abspath(self.cache_path)), exist_ok=True)
            with open(self.cache_path, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)

    def tile_patches(self, problems, precision=B.FP32) -> list:
        """Patches per tile for each problem (a list of Scene-like objects
        with n_frames, n_patches, n_edges); tunes buckets not in the cache."""
        buckets = [bucket_of(s.n_frames, s.n_patches, s.n_edges) for s in problems]
        for bk in sorted(set(buckets)):
            key = self._key(bk, precision)
            if key not in self.table:
                members = [s for s, b in zip(problems, buckets) if b == bk][: self.members]
                self.table[key] = self._tune(members, precision)
        self.save()
        return [int(self.table[self._key(bk, precision)]["best"]) for bk in buckets]

    def _tune(self, members, precision) -> dict:
        ctx = B.Context(0)
        batch = B.BatchTensors.from_scenes(members)
        dt = torch.float64 if precision == B.FP64 else torch.float32
        times = {}
        stream = torch.cuda.current_stream()
        for K in self.candidates:
            try:
                ctx.analyze_batch(batch, [K] * len(members))
            except B.DpvbaError:
                continue  # a tile of this size does not fit
            poses0 = batch.poses.to(dt)
            depth0 = batch.inv_depth.to(dt)
            poses, depth = poses0.clone(), depth0.clone()
            ctx.solve_batch(batch, poses, depth, n_iters=2, precision=precision, report=False)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(self.steps):
                poses.copy_(poses0)
                depth.copy_(depth0)
                ctx.solve_batch(batch, poses, depth, n_iters=2, precision=precision, report=False)
            ev1.record(stream)
            ev1.synchronize()
            times[K] = ev0.elapsed_time(ev1) / self.steps
        ctx.close()
        best = min(times, key=times.get)
        return {"best": int(best), "ms": {str(k): round(v, 4) for k, v in times.items()}}
