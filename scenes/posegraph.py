"""Seeded pose graphs for the Sim(3) pose-graph optimisation of the
classical loop closure: a ground-truth trajectory, a drifted estimate (scale
and heading drift accumulated along the odometry) and loop measurements
DeltaS^loop_jk taken from the ground truth, stated so that the loop term
log(DeltaS^loop_jk S_j^-1 S_k) vanishes at the ground truth.  World
simulation only: 4 x 4 matrices, no optimisation arithmetic."""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


def _pose(R, c):
    q = Rotation.from_matrix(R).as_quat()
    q *= np.where(q[:, 3:4] < 0, -1.0, 1.0)
    return np.concatenate([c, q], 1)


def _mat(R, c):
    M = np.tile(np.eye(4), (R.shape[0], 1, 1))
    M[:, :3, :3] = R
    M[:, :3, 3] = c
    return M


def loop_problem(n=40, seed=0, drift=0.05, heading=0.02, loops=None, radius=5.0, turns=0.95):
    """(poses0 [n,7], poses_gt [n,7], loop_j, loop_k, loop_rel [L,8] (t, q, s))."""
    rng = np.random.default_rng(seed)
    ang = np.linspace(0.0, 2 * np.pi * turns, n)
    c_gt = np.stack([radius * np.cos(ang), radius * np.sin(ang), 0.1 * rng.normal(size=n)], 1)
    R_gt = Rotation.from_euler("z", ang + np.pi / 2).as_matrix()
    steps = np.diff(c_gt, axis=0) * (1 + drift * np.arange(1, n)[:, None] / n)
    c0 = np.concatenate([c_gt[:1], c_gt[0] + np.cumsum(steps, 0)], 0)
    R0 = Rotation.from_euler("z", ang + np.pi / 2 + heading * np.arange(n) / n).as_matrix()
    if loops is None:
        loops = [(i, n - 1 - i) for i in range(0, n // 4, max(1, n // 20))]
    lj = np.array([a for a, _ in loops], dtype=np.int32)
    lk = np.array([b for _, b in loops], dtype=np.int32)
    M = _mat(R_gt, c_gt)
    # DeltaS^loop_jk = (S_j^-1 S_k)^-1 = S_k^-1 S_j at the ground truth (scale 1)
    D = np.linalg.inv(M[lk]) @ M[lj]
    loop_rel = np.concatenate([_pose(D[:, :3, :3], D[:, :3, 3]), np.ones((len(lj), 1))], 1)
    return _pose(R0, c0), _pose(R_gt, c_gt), lj, lk, loop_rel
