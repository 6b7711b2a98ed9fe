"""SO(3) / SE(3) helpers in float64 for the oracle.

Test infrastructure only (see the package docstring).

Conventions: quaternions are (x, y, z, w); a pose is camera-to-world
(t, q); perturbations act on the right, G <- G * Exp(xi) with xi = (rho, phi),
rho the translational and phi the rotational part.
"""
from __future__ import annotations

import numpy as np


def hat(v: np.ndarray) -> np.ndarray:
    """Skew matrix [v]_x with [v]_x w = v x w; works on [..., 3]."""
    v = np.asarray(v, dtype=np.float64)
    O = np.zeros(v.shape[:-1] + (3, 3))
    O[..., 0, 1] = -v[..., 2]
    O[..., 0, 2] = v[..., 1]
    O[..., 1, 0] = v[..., 2]
    O[..., 1, 2] = -v[..., 0]
    O[..., 2, 0] = -v[..., 1]
    O[..., 2, 1] = v[..., 0]
    return O


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of a (normalised) quaternion (x, y, z, w)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - z * w)
    R[..., 0, 2] = 2 * (x * z + y * w)
    R[..., 1, 0] = 2 * (x * y + z * w)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - x * w)
    R[..., 2, 0] = 2 * (x * z - y * w)
    R[..., 2, 1] = 2 * (y * z + x * w)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rot_to_quat(R: np.ndarray) -> np.ndarray:
    """Quaternion (x, y, z, w), w >= 0, of rotation matrices (Shepperd's method:
    pick the largest of the four squared components to divide by)."""
    R = np.asarray(R, dtype=np.float64)
    flat = R.reshape(-1, 3, 3)
    out = np.empty((flat.shape[0], 4))
    for n, M in enumerate(flat):
        tr = M[0, 0] + M[1, 1] + M[2, 2]
        cand = np.array([M[0, 0], M[1, 1], M[2, 2], tr])
        m = int(np.argmax(cand))
        if m == 3:
            s = 2.0 * np.sqrt(1.0 + tr)
            q = [(M[2, 1] - M[1, 2]) / s, (M[0, 2] - M[2, 0]) / s, (M[1, 0] - M[0, 1]) / s, 0.25 * s]
        elif m == 0:
            s = 2.0 * np.sqrt(1.0 + M[0, 0] - M[1, 1] - M[2, 2])
            q = [0.25 * s, (M[0, 1] + M[1, 0]) / s, (M[0, 2] + M[2, 0]) / s, (M[2, 1] - M[1, 2]) / s]
        elif m == 1:
            s = 2.0 * np.sqrt(1.0 + M[1, 1] - M[0, 0] - M[2, 2])
            q = [(M[0, 1] + M[1, 0]) / s, 0.25 * s, (M[1, 2] + M[2, 1]) / s, (M[0, 2] - M[2, 0]) / s]
        else:
            s = 2.0 * np.sqrt(1.0 + M[2, 2] - M[0, 0] - M[1, 1])
            q = [(M[0, 2] + M[2, 0]) / s, (M[1, 2] + M[2, 1]) / s, 0.25 * s, (M[1, 0] - M[0, 1]) / s]
        q = np.asarray(q)
        q /= np.linalg.norm(q)
        out[n] = -q if q[3] < 0 else q
    return out.reshape(R.shape[:-2] + (4,))


# Below this squared angle the trigonometric coefficients are replaced by
# their Taylor series (error O(theta^4) relative, below float64 rounding).
SMALL_THETA2 = 1e-10


def _coeffs(phi: np.ndarray):
    """A = sin t / t, B = (1 - cos t) / t^2, C = (t - sin t) / t^3 with t = |phi|."""
    th2 = np.sum(phi * phi, axis=-1)
    small = th2 < SMALL_THETA2
    th = np.sqrt(np.where(small, 1.0, th2))
    A = np.where(small, 1.0 - th2 / 6.0, np.sin(th) / th)
    B = np.where(small, 0.5 - th2 / 24.0, (1.0 - np.cos(th)) / np.where(small, 1.0, th2))
    C = np.where(small, 1.0 / 6.0 - th2 / 120.0, (th - np.sin(th)) / (th * np.where(small, 1.0, th2)))
    return A, B, C


def so3_exp(phi: np.ndarray) -> np.ndarray:
    """Rodrigues: Exp(phi) = I + A [phi]_x + B [phi]_x^2."""
    phi = np.asarray(phi, dtype=np.float64)
    A, B, _ = _coeffs(phi)
    K = hat(phi)
    I = np.broadcast_to(np.eye(3), K.shape)
    return I + A[..., None, None] * K + B[..., None, None] * (K @ K)


def so3_left_jacobian(phi: np.ndarray) -> np.ndarray:
    """V(phi) = I + B [phi]_x + C [phi]_x^2, the translational coupling of SE(3) Exp."""
    phi = np.asarray(phi, dtype=np.float64)
    _, B, C = _coeffs(phi)
    K = hat(phi)
    I = np.broadcast_to(np.eye(3), K.shape)
    return I + B[..., None, None] * K + C[..., None, None] * (K @ K)


def se3_exp(xi: np.ndarray):
    """SE(3) Exp of xi = (rho, phi): rotation Exp(phi), translation V(phi) rho."""
    xi = np.asarray(xi, dtype=np.float64)
    rho, phi = xi[..., :3], xi[..., 3:]
    return so3_exp(phi), np.einsum("...ab,...b->...a", so3_left_jacobian(phi), rho)


def so3_log(R: np.ndarray) -> np.ndarray:
    """Rotation vector of R (angle in [0, pi])."""
    R = np.asarray(R, dtype=np.float64)
    cos = np.clip((np.trace(R, axis1=-2, axis2=-1) - 1.0) / 2.0, -1.0, 1.0)
    th = np.arccos(cos)
    v = np.stack([R[..., 2, 1] - R[..., 1, 2], R[..., 0, 2] - R[..., 2, 0], R[..., 1, 0] - R[..., 0, 1]], axis=-1)
    s = np.sin(th)
    small = th < 1e-6
    factor = np.where(small, 0.5 + th * th / 12.0, th / (2.0 * np.where(small, 1.0, s)))
    out = factor[..., None] * v
    near_pi = th > np.pi - 1e-6
    if np.any(near_pi):
        for idx in zip(*np.nonzero(near_pi)) if R.ndim > 2 else [()]:
            M = R[idx]
            a = int(np.argmax(np.diag(M)))
            col = (M[:, a] + np.eye(3)[:, a]) / np.sqrt(2.0 * (1.0 + M[a, a]))
            out[idx] = np.pi * col
    return out


def pose_to_rt(poses: np.ndarray):
    """(R, t) of camera-to-world poses [..., 7] = (t, q)."""
    poses = np.asarray(poses, dtype=np.float64)
    return quat_to_rot(poses[..., 3:7]), poses[..., :3].copy()


def rt_to_pose(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.concatenate([t, rot_to_quat(R)], axis=-1)


def retract_right(R: np.ndarray, t: np.ndarray, xi: np.ndarray):
    """G * Exp(xi): R <- R Exp(phi), t <- t + R V(phi) rho."""
    dR, dt = se3_exp(xi)
    return R @ dR, t + np.einsum("...ab,...b->...a", R, dt)
