"""Seeded synthetic scenes shaped like the paper's patch graphs (Sec. 3.1-3.2).

Geometry conventions (shared by every consumer, fixed here once):

* A pose is camera-to-world, stored as ``(tx, ty, tz, qx, qy, qz, qw)``: the
  camera centre in world coordinates and the unit quaternion of the rotation
  that maps camera axes to world axes.
* Camera axes: x right, y down, z forward.  Pinhole ``fx = fy = 320``,
  ``cx = 320``, ``cy = 240`` on a 640x480 image.
* A patch is ``p x p`` pixels (p = 3) around a centre drawn uniformly in
  ``[8, 632] x [8, 472]``, with one inverse depth drawn from ``U[0.2, 2]``.
  ``patches[k, a, b] = (u + b - c, v + a - c)`` with ``c = (p - 1) / 2``.
* Edges ``(i, k, j)`` run from patch ``k`` (owned by frame ``i``) to frame ``j``
  and are emitted sorted by (source frame, patch, target frame).
* Targets are the world point rendered into frame ``j`` plus ``N(0, 0.5^2)``
  pixel noise per axis; weights are drawn from ``U(0.1, 1]`` per axis.
* A patch is redrawn until every one of its edges sees its world point at
  camera depth >= 0.2 (twice the validity threshold the solver uses).

Random streams: ``Generator(PCG64(SeedSequence([1000 * cfg + instance, stream])))``
with stream 0 for the scene and stream 1 for the initial estimate.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np
from scipy.spatial.transform import Rotation

FX = FY = 320.0
CX, CY = 320.0, 240.0
IMG_W, IMG_H = 640, 480
PATCH = 3
MIN_REAL_DEPTH = 0.2

CONFIG_NAMES = {
    0: "cfg0_allpairs_8x96",
    1: "cfg1_window_22x96_r13",
    2: "cfg2_global_1000x96_loop",
    3: "cfg3_adjoint_16_windows",
    4: "cfg4_batched_256",
}


def _rng(cfg: int, instance: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1000 * cfg + instance, stream])))


@dataclass
class Scene:
    """One BA problem: inputs (float32 / int32) plus float64 ground truth."""

    name: str
    n_frames: int
    n_fixed: int
    poses: np.ndarray          # [N,7] float32, initial estimate
    patches: np.ndarray        # [P,p,p,2] float32
    inv_depth: np.ndarray      # [P] float32, initial estimate
    ii: np.ndarray             # [E] int32 source frame
    jj: np.ndarray             # [E] int32 target frame
    kk: np.ndarray             # [E] int32 patch
    target: np.ndarray         # [E,2] float32
    weight: np.ndarray         # [E,2] float32
    intrinsics: np.ndarray     # [4] float32 (fx, fy, cx, cy)
    poses_gt: np.ndarray       # [N,7] float64
    inv_depth_gt: np.ndarray   # [P] float64
    target64: np.ndarray       # [E,2] float64 targets before rounding to float32
    n_iters: int = 2
    lam: float = 1e-4
    z_min: float = 0.1
    meta: dict = field(default_factory=dict)

    @property
    def n_patches(self) -> int:
        return int(self.inv_depth.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.ii.shape[0])

    @property
    def patch_size(self) -> int:
        return int(self.patches.shape[1])


# ----------------------------------------------------------------------------
# trajectories: rotations R_cw [N,3,3] and centres c [N,3], float64
# ----------------------------------------------------------------------------

def _yaw_matrix(psi: np.ndarray) -> np.ndarray:
    """Camera-to-world rotation of a camera whose forward axis has heading psi
    about the world y (down) axis."""
    c, s = np.cos(psi), np.sin(psi)
    R = np.zeros(psi.shape + (3, 3))
    R[..., 0, 0] = c
    R[..., 0, 2] = s
    R[..., 1, 1] = 1.0
    R[..., 2, 0] = -s
    R[..., 2, 2] = c
    return R


def random_walk_trajectory(rng: np.random.Generator, n: int, step: float = 0.1,
                           yaw_sigma_deg: float = 2.0):
    """Random walk: fixed-length steps in uniformly random directions, yaw
    jitter about the camera y axis per step; frame 0 at the identity."""
    R = np.zeros((n, 3, 3))
    c = np.zeros((n, 3))
    R[0] = np.eye(3)
    for m in range(1, n):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c[m] = c[m - 1] + step * d
        yaw = np.deg2rad(rng.normal(0.0, yaw_sigma_deg))
        R[m] = R[m - 1] @ _yaw_matrix(np.array(yaw))
    return R, c


def forward_trajectory(n: int, phase: float = 0.0, speed: float = 0.02):
    """Smooth forward motion along the optical axis with a slow yaw swing
    (5 deg * sin(2 pi t / 200)) and a small vertical sway."""
    t = np.arange(n, dtype=np.float64) + phase
    psi = np.deg2rad(5.0) * np.sin(2.0 * np.pi * t / 200.0)
    R = _yaw_matrix(psi)
    fwd = np.stack([np.sin(psi), np.zeros_like(psi), np.cos(psi)], axis=1)
    c = np.zeros((n, 3))
    c[1:] = np.cumsum(speed * fwd[:-1], axis=0)
    c[:, 1] = 0.01 * np.sin(2.0 * np.pi * t / 50.0)
    return R, c


def circle_trajectory(n: int = 1000, radius: float = 20.0, laps: float = 1.58):
    """Closed-loop circle traversed ``laps`` times; the camera looks
    horizontally at the circle centre."""
    theta = 2.0 * np.pi * laps * np.arange(n) / n
    c = np.stack([radius * np.cos(theta), np.zeros(n), radius * np.sin(theta)], axis=1)
    psi = np.arctan2(-np.cos(theta), -np.sin(theta))
    return _yaw_matrix(psi), c


# ----------------------------------------------------------------------------
# rendering
# ----------------------------------------------------------------------------

def _world_points(R, c, f, u, v, d):
    """World points of pixels (u, v) with inverse depth d seen from frame f."""
    ray = np.stack([(u - CX) / FX, (v - CY) / FY, np.ones_like(u)], axis=-1)
    Xc = ray / d[:, None]
    return Xc @ R[f].T + c[f]


def _camera_points(R, c, g, Xw):
    """World points expressed in camera g (world-to-camera = R_g^T (X - c_g))."""
    return (Xw - c[g]) @ R[g]


def _render(Xg):
    return np.stack([FX * Xg[..., 0] / Xg[..., 2] + CX, FY * Xg[..., 1] / Xg[..., 2] + CY], axis=-1)


def _draw_patches(rng, R, c, f, n_patch, targets):
    """Draw patch centres and inverse depths for frame f, redrawing any patch
    whose world point would sit at camera depth < MIN_REAL_DEPTH in a target."""
    f32 = lambda x: x.astype(np.float32).astype(np.float64)  # store exactly what is rendered
    u = f32(rng.uniform(8.0, IMG_W - 8.0, size=n_patch))
    v = f32(rng.uniform(8.0, IMG_H - 8.0, size=n_patch))
    d = f32(rng.uniform(0.2, 2.0, size=n_patch))
    for _attempt in range(1000):
        Xw = _world_points(R, c, f, u, v, d)
        bad = np.zeros(n_patch, dtype=bool)
        for g in targets:
            bad |= _camera_points(R, c, g, Xw)[:, 2] < MIN_REAL_DEPTH
        if not bad.any():
            return u, v, d, Xw
        nb = int(bad.sum())
        u[bad] = f32(rng.uniform(8.0, IMG_W - 8.0, size=nb))
        v[bad] = f32(rng.uniform(8.0, IMG_H - 8.0, size=nb))
        d[bad] = f32(rng.uniform(0.2, 2.0, size=nb))
    raise RuntimeError("could not place patches in front of all target cameras")


def _patch_grid(u, v, p):
    r = np.arange(p, dtype=np.float64) - (p - 1) / 2
    P = np.empty((u.shape[0], p, p, 2))
    P[..., 0] = u[:, None, None] + r[None, None, :]
    P[..., 1] = v[:, None, None] + r[None, :, None]
    return P


def _pose_array(R, c):
    q = Rotation.from_matrix(R).as_quat()  # (x, y, z, w)
    q *= np.where(q[:, 3:4] < 0, -1.0, 1.0)
    return np.concatenate([c, q], axis=1)


def _render_graph(rng, R, c, patches_per_frame, targets_of, noise_px):
    """Patches, edges (sorted by source frame, patch, target), targets, weights."""
    n = R.shape[0]
    U, V, D = [], [], []
    ii, jj, kk, tgt = [], [], [], []
    k0 = 0
    for f in range(n):
        tf = np.asarray(sorted(targets_of(f)), dtype=np.int64)
        K = int(patches_per_frame[f])
        u, v, d, Xw = _draw_patches(rng, R, c, f, K, tf)
        U.append(u); V.append(v); D.append(d)
        if tf.size:
            proj = np.stack([_render(_camera_points(R, c, g, Xw)) for g in tf], axis=1)  # [K,T,2]
            ii.append(np.full(K * tf.size, f))
            jj.append(np.tile(tf, K))
            kk.append(np.repeat(np.arange(k0, k0 + K), tf.size))
            tgt.append(proj.reshape(-1, 2))
        k0 += K
    u = np.concatenate(U); v = np.concatenate(V); d = np.concatenate(D)
    ii = np.concatenate(ii); jj = np.concatenate(jj); kk = np.concatenate(kk)
    tgt = np.concatenate(tgt)
    E = ii.shape[0]
    tgt = tgt + rng.normal(0.0, noise_px, size=(E, 2)) if noise_px > 0 else tgt
    w = 1.0 - rng.uniform(0.0, 0.9, size=(E, 2))   # U(0.1, 1]
    return u, v, d, ii, jj, kk, tgt, w


def _perturbed_init(rng, R, c, d, n_fixed, rho_sigma=0.01, phi_sigma_deg=0.5, logd_sigma=0.05):
    """Free poses: R_gt * Rot(phi), c_gt + rho; inverse depth d_gt * exp(eps).
    Poses [0, n_fixed) start at ground truth."""
    n = R.shape[0]
    R0 = R.copy(); c0 = c.copy()
    free = np.arange(n_fixed, n)
    if free.size:
        phi = np.deg2rad(phi_sigma_deg) * rng.normal(size=(free.size, 3))
        R0[free] = R[free] @ Rotation.from_rotvec(phi).as_matrix()
        c0[free] = c[free] + rho_sigma * rng.normal(size=(free.size, 3))
    d0 = d * np.exp(logd_sigma * rng.normal(size=d.shape))
    return R0, c0, d0


def _assemble_scene(name, R, c, u, v, d, ii, jj, kk, tgt, w, n_fixed, R0, c0, d0,
                    n_iters, lam, meta=None):
    return Scene(
        name=name, n_frames=R.shape[0], n_fixed=n_fixed,
        poses=_pose_array(R0, c0).astype(np.float32),
        patches=_patch_grid(u, v, PATCH).astype(np.float32),
        inv_depth=d0.astype(np.float32),
        ii=ii.astype(np.int32), jj=jj.astype(np.int32), kk=kk.astype(np.int32),
        target=tgt.astype(np.float32), weight=w.astype(np.float32),
        intrinsics=np.array([FX, FY, CX, CY], dtype=np.float32),
        poses_gt=_pose_array(R, c), inv_depth_gt=d.astype(np.float64),
        target64=tgt.astype(np.float64),
        n_iters=n_iters, lam=lam, meta=dict(meta or {}),
    )


def _window_targets(n, radius):
    return lambda f: [g for g in range(max(0, f - radius), min(n, f + radius + 1)) if g != f]


# ----------------------------------------------------------------------------
# public constructors
# ----------------------------------------------------------------------------

def tiny_scene(n_frames=4, patches_per_frame=6, seed=0, radius=None, n_fixed=2,
               noise_px=0.5, init="perturb", trajectory="walk") -> Scene:
    """Small scene for brute-force checks.  ``init`` is "perturb" or "gt"."""
    rng = _rng(9, seed, 0)
    if trajectory == "walk":
        R, c = random_walk_trajectory(rng, n_frames)
    else:
        R, c = forward_trajectory(n_frames)
    radius = n_frames if radius is None else radius
    u, v, d, ii, jj, kk, tgt, w = _render_graph(
        rng, R, c, [patches_per_frame] * n_frames, _window_targets(n_frames, radius), noise_px)
    if init == "gt":
        R0, c0, d0 = R, c, d
    else:
        R0, c0, d0 = _perturbed_init(_rng(9, seed, 1), R, c, d, n_fixed)
    return _assemble_scene(f"tiny_{n_frames}x{patches_per_frame}_s{seed}", R, c, u, v, d,
                           ii, jj, kk, tgt, w, n_fixed, R0, c0, d0, n_iters=2, lam=1e-4)


def _cfg0(noise_px=0.5):
    rng = _rng(0, 0, 0)
    R, c = random_walk_trajectory(rng, 8, step=0.1, yaw_sigma_deg=2.0)
    u, v, d, ii, jj, kk, tgt, w = _render_graph(rng, R, c, [96] * 8, _window_targets(8, 8), noise_px)
    R0, c0, d0 = _perturbed_init(_rng(0, 0, 1), R, c, d, 2)
    return _assemble_scene(CONFIG_NAMES[0], R, c, u, v, d, ii, jj, kk, tgt, w, 2, R0, c0, d0,
                           n_iters=2, lam=1e-4)


WINDOW = 22
WINDOW_RADIUS = 13
WINDOW_FREE = 12
N_CALLS = 1000


@lru_cache(maxsize=2)
def window_sequence(n_calls: int = N_CALLS, noise_px: float = 0.5):
    """The global forward trajectory behind the sliding-window workload: frames,
    patches and every edge within +-13 frames, rendered once."""
    n = n_calls + WINDOW - 1
    rng = _rng(1, 0, 0)
    R, c = forward_trajectory(n)
    u, v, d, ii, jj, kk, tgt, w = _render_graph(rng, R, c, [96] * n, _window_targets(n, WINDOW_RADIUS), noise_px)
    return dict(R=R, c=c, u=u, v=v, d=d, ii=ii, jj=jj, kk=kk, tgt=tgt, w=w, K=96)


def make_window(call: int, n_calls: int = N_CALLS, noise_px: float = 0.5) -> Scene:
    """Window ``call`` of the sliding-window workload: frames [call, call+22),
    last 12 poses free, edges within +-13 frames inside the window.  Local
    indices (frame 0 = first frame of the window), so every window has the
    same (ii, jj, kk)."""
    seq = window_sequence(n_calls, noise_px)
    K = seq["K"]
    f0, f1 = call, call + WINDOW
    # the global edge list is sorted by source frame: slice that range first
    e0, e1 = np.searchsorted(seq["ii"], [f0, f1])
    sel = e0 + np.nonzero((seq["jj"][e0:e1] >= f0) & (seq["jj"][e0:e1] < f1))[0]
    R = seq["R"][f0:f1]; c = seq["c"][f0:f1]
    p0, p1 = f0 * K, f1 * K
    u = seq["u"][p0:p1]; v = seq["v"][p0:p1]; d = seq["d"][p0:p1]
    ii = seq["ii"][sel] - f0; jj = seq["jj"][sel] - f0; kk = seq["kk"][sel] - p0
    n_fixed = WINDOW - WINDOW_FREE
    R0, c0, d0 = _perturbed_init(_rng(1, call, 1), R, c, d, n_fixed)
    return _assemble_scene(f"{CONFIG_NAMES[1]}_call{call}", R, c, u, v, d, ii, jj, kk,
                           seq["tgt"][sel], seq["w"][sel], n_fixed, R0, c0, d0, n_iters=2, lam=1e-4,
                           meta={"call": call})


def _loop_targets(c, min_gap=100, max_dist=2.0, n_loop=10):
    n = c.shape[0]
    D = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=-1)
    loops = []
    for i in range(n):
        cand = np.arange(i + min_gap + 1, n)
        cand = cand[D[i, cand] < max_dist]
        order = np.lexsort((cand, D[i, cand]))  # nearest first, ties -> lower j
        loops.append(sorted(cand[order[:n_loop]].tolist()))
    return loops


CFG2_DRIFT = 0.02   # linear scale drift reached at the last keyframe


def _cfg2(noise_px=0.5, n_frames=1000, drift=CFG2_DRIFT, patches_per_frame=96, name=None):
    rng = _rng(2, 0, 0)
    R, c = circle_trajectory(n_frames)
    loops = _loop_targets(c)
    temporal = _window_targets(n_frames, 6)
    targets_of = lambda f: sorted(set(temporal(f)) | set(loops[f]))
    K = patches_per_frame
    u, v, d, ii, jj, kk, tgt, w = _render_graph(rng, R, c, [K] * n_frames, targets_of, noise_px)
    # initial estimate with scale drift: steps scaled by s_n, depths divided by s_n
    rng1 = _rng(2, 0, 1)
    s = 1.0 + drift * np.arange(n_frames) / (n_frames - 1)
    c0 = np.zeros_like(c)
    c0[0] = c[0]
    for m in range(1, n_frames):
        c0[m] = c0[m - 1] + s[m] * (c[m] - c[m - 1])
    phi = np.deg2rad(0.1) * rng1.normal(size=(n_frames, 3))
    phi[0] = 0.0
    R0 = R @ Rotation.from_rotvec(phi).as_matrix()
    d0 = d / np.repeat(s, K)
    return _assemble_scene(CONFIG_NAMES[2] if name is None else name, R, c, u, v, d, ii, jj, kk, tgt, w, 1, R0,
                           c0, d0, n_iters=5, lam=1e-4, meta={"loop_pairs": int(sum(len(x) for x in loops))})


def relabel_frames(s: Scene, seed: int = 0) -> Scene:
    """The same problem with its free frames numbered in a random order (the
    fixed frames keep the first indices): frame f becomes new[f].  A banded
    graph turns into one whose frame order couples distant indices, the case
    a fill-reducing order of the reduced system has to undo."""
    rng = np.random.default_rng(seed)
    nf, N = s.n_fixed, s.n_frames
    new = np.r_[np.arange(nf), nf + rng.permutation(N - nf)].astype(np.int32)
    out = Scene(**{k: getattr(s, k) for k in s.__dataclass_fields__})
    out.name = f"{s.name}_relabelled{seed}"
    out.poses = np.empty_like(s.poses)
    out.poses[new] = s.poses
    out.poses_gt = np.empty_like(s.poses_gt)
    out.poses_gt[new] = s.poses_gt
    out.ii = new[s.ii]
    out.jj = new[s.jj]
    out.meta = dict(s.meta, relabel=new)
    return out


def make_sweep(n_frames: int, total_patches: int = 96000, noise_px: float = 0.5) -> Scene:
    """Keyframe-count sweep of the global BA (the synthetic analogue of the
    paper's BA-size study, Appendix A): n_frames keyframes on the same circle
    (1.58 laps), the total number of patches held at ``total_patches``
    (total_patches / n_frames per frame), +-6 temporal targets and the same
    proximity loop rule as the 1000-keyframe workload (about 12-16 edges per
    patch), 2 % scale drift, the first pose fixed, 5 GN iterations.
    make_sweep(1000) is the 1000-keyframe workload itself."""
    K = total_patches // n_frames
    return _cfg2(noise_px, n_frames=n_frames, patches_per_frame=K,
                 name=CONFIG_NAMES[2] if (n_frames, K) == (1000, 96) else f"sweep_{n_frames}x{K}")


def _cfg_window_instance(cfg, b, F, K, radius, n_fixed, noise_px=0.5):
    rng = _rng(cfg, b, 0)
    phase = float(rng.uniform(0.0, 200.0))
    R, c = forward_trajectory(F, phase=phase)
    u, v, d, ii, jj, kk, tgt, w = _render_graph(rng, R, c, [K] * F, _window_targets(F, radius), noise_px)
    R0, c0, d0 = _perturbed_init(_rng(cfg, b, 1), R, c, d, n_fixed)
    return _assemble_scene(f"{CONFIG_NAMES[cfg]}_{b}", R, c, u, v, d, ii, jj, kk, tgt, w,
                           n_fixed, R0, c0, d0, n_iters=2, lam=1e-4,
                           meta={"F": F, "K": K, "radius": radius})


def instance_shapes(cfg: int, count: int):
    """(F, K, radius, n_fixed) per instance of the batched workloads."""
    rng = _rng(cfg, 0, 2)
    out = []
    for _ in range(count):
        if cfg == 3:
            F = int(rng.integers(12, 23)); K = int(rng.integers(64, 97)); r = WINDOW_RADIUS
            out.append((F, K, r, max(2, F - WINDOW_FREE)))
        else:
            F = int(rng.integers(8, 41)); K = int(rng.integers(48, 129)); r = int(rng.integers(4, 14))
            out.append((F, K, r, 2))
    return out


def make_config(cfg: int, instance: int = 0, noise_px: float = 0.5) -> Scene:
    if cfg == 0:
        return _cfg0(noise_px)
    if cfg == 1:
        return make_window(instance, noise_px=noise_px)
    if cfg == 2:
        return _cfg2(noise_px)
    if cfg in (3, 4):
        count = 16 if cfg == 3 else 256
        F, K, r, nf = instance_shapes(cfg, count)[instance]
        return _cfg_window_instance(cfg, instance, F, K, r, nf, noise_px)
    raise ValueError(f"unknown config {cfg}")
