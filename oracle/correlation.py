"""Patch correlation of DPV-SLAM eq. 4 -- test infrastructure.

Only tests/ and bench.py's CPU-baseline leg use this module; the product
path never imports it.

Sec. 3.1, "Patch correlation": for an edge (i, k, j) the patch P_k is
reprojected into frame j (eq. 2) and, at every patch pixel (u, v), the patch
feature vector g(u, v) is dotted with the frame-j feature map f sampled
bilinearly at the reprojected point shifted by every offset of a 7 x 7 grid
centred at zero:
    C(u, v, a, b) = < g(u, v), f(P'(u, v) + Delta_ab) >.

Readings where the paper is silent:
  * Delta_ab = (a - 3, b - 3) added to (x, y); C is stored [E, p, p, 7, 7]
    with (u, v) = (patch row, patch column);
  * coordinates are in feature-map pixels, pixel (x, y) holding the value of
    map[y, x]; bilinear sampling weighs the four pixels around the point by
    their distances, pixels outside the map count as zero;
  * feature maps are [frames, H, W, D] and patch features [P, p, p, D].
Float64 throughout, from the float32 inputs promoted exactly.
"""
from __future__ import annotations

import numpy as np

RADIUS = 3          # the 7 x 7 grid of offsets -3 .. 3
GRID = 2 * RADIUS + 1


def bilinear(fmap: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Feature vectors [..., D] of one map [H, W, D] at points (x, y) [...],
    zero outside."""
    H, W, D = fmap.shape
    # points farther out than any map are outside either way; the clip only
    # keeps the integer conversion defined
    x = np.clip(x, -1e9, 1e9)
    y = np.clip(y, -1e9, 1e9)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx = x - x0
    fy = y - y0
    out = np.zeros(x.shape + (D,))
    for dy, wy in ((0, 1.0 - fy), (1, fy)):
        for dx, wx in ((0, 1.0 - fx), (1, fx)):
            xi, yi = x0 + dx, y0 + dy
            inside = (xi >= 0) & (xi < W) & (yi >= 0) & (yi < H)
            v = fmap[np.clip(yi, 0, H - 1), np.clip(xi, 0, W - 1)].astype(np.float64)
            out += (wx * wy * inside)[..., None] * v
    return out


def correlation(gmap, fmaps, kk, jj, coords):
    """C [E, p, p, 7, 7] of eq. 4.  gmap [P, p, p, D], fmaps [M, H, W, D],
    kk / jj [E] (patch, feature map of the target frame), coords
    [E, p, p, 2] reprojected (x, y) in feature-map pixels."""
    gmap = np.asarray(gmap, dtype=np.float64)
    coords = np.asarray(coords, dtype=np.float64)
    E, p = coords.shape[0], coords.shape[1]
    off = np.arange(GRID) - RADIUS
    C = np.zeros((E, p, p, GRID, GRID))
    for e in range(E):
        f = fmaps[int(jj[e])]
        g = gmap[int(kk[e])]                                       # [p, p, D]
        x = coords[e, :, :, 0][:, :, None, None] + off[None, None, :, None]
        y = coords[e, :, :, 1][:, :, None, None] + off[None, None, None, :]
        x, y = np.broadcast_arrays(x, y)                           # [p, p, 7, 7]
        C[e] = np.einsum("uvabd,uvd->uvab", bilinear(f, x, y), g)
    return C
