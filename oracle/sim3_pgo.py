"""Sim(3) pose-graph optimisation of the classical loop closure -- test
infrastructure.

Only tests/ and bench.py's CPU-baseline leg use this module; the product
path never imports it.

DPV-SLAM Sec. 3.3 ("Optimization"): every keyframe i gets an absolute
similarity S_i in Sim(3), initialised from its current pose with scale 1.
The relative similarities marked Delta are constants.  A smoothness term
links each keyframe to its successor (eq. 5),
    r_i = log(DeltaS_(i,i+1)^-1 S_i^-1 S_(i+1)),
each detected loop (j, k) contributes (eq. 6)
    r_jk = log(DeltaS^loop_jk S_j^-1 S_k),
and sum_i |r_i|^2 + sum_(j,k) |r_jk|^2 (eq. 7) is minimised by
Levenberg-Marquardt.  Afterwards G_i <- (t_i, R_i) and d_i <- d_i / s_i.

Readings where the paper is silent:
  * S = (R, t, s) maps x to s R x + t; S_a S_b = (R_a R_b, s_a R_a t_b + t_a,
    s_a s_b); a pose (t, q) becomes (R(q), t, 1);
  * DeltaS_(i,i+1) = S_i^-1 S_(i+1) of the initial similarities, so the
    smoothness terms start at zero and keep the odometry's relative motion;
  * tangent coordinates xi = (rho, phi, sigma): translation, rotation,
    log-scale; Exp(xi) = expm of the 4x4 generator [[sigma I + [phi]x, rho],
    [0, 0]], log its inverse near the identity;
  * right perturbations S <- S Exp(delta); the first n_fixed similarities
    are held (the objective is invariant to a global similarity);
  * Levenberg-Marquardt with H~ = H + lambda (Diag(H) + I), a fixed lambda,
    a fixed number of iterations and no step rejection, as for the BA.
Float64 throughout.  Jacobians of the residuals are taken by torch autograd
through the definition (torch.linalg.matrix_exp), so they are exact.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def _eye(n):
    return torch.eye(n, dtype=F64)


def hat(v):
    z = torch.zeros(v.shape[:-1], dtype=v.dtype)
    return torch.stack([torch.stack([z, -v[..., 2], v[..., 1]], -1),
                        torch.stack([v[..., 2], z, -v[..., 0]], -1),
                        torch.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def quat_to_rot(q):
    """Rotation matrices of unit quaternions (x, y, z, w) [..., 4]."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    x, y, z, w = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], -2)


def rot_to_quat(R):
    """Unit quaternions (x, y, z, w) with w >= 0 of rotation matrices (numpy)."""
    from scipy.spatial.transform import Rotation
    q = Rotation.from_matrix(np.asarray(R)).as_quat()
    return q * np.where(q[..., 3:4] < 0, -1.0, 1.0)


def _w_matrix(phi, sigma):
    """W(phi, sigma) = int_0^1 exp(tau (sigma I + [phi]x)) dtau, the top-right
    block of expm([[M, I], [0, 0]]) with M = sigma I + [phi]x."""
    M = sigma[..., None, None] * _eye(3) + hat(phi)
    Z = torch.zeros(M.shape[:-2] + (6, 6), dtype=F64)
    Z[..., :3, :3] = M
    Z[..., :3, 3:] = _eye(3)
    return torch.linalg.matrix_exp(Z)[..., :3, 3:]


def exp(xi):
    """(R, t, s) of Exp(xi), xi = (rho, phi, sigma) [..., 7]."""
    rho, phi, sigma = xi[..., :3], xi[..., 3:6], xi[..., 6]
    R = torch.linalg.matrix_exp(hat(phi))
    t = (_w_matrix(phi, sigma) @ rho[..., None])[..., 0]
    return R, t, torch.exp(sigma)


def so3_log(R):
    """phi with expm([phi]x) = R for rotation angles below pi."""
    v = 0.5 * torch.stack([R[..., 2, 1] - R[..., 1, 2], R[..., 0, 2] - R[..., 2, 0], R[..., 1, 0] - R[..., 0, 1]], -1)
    s2 = (v * v).sum(-1)
    c = 0.5 * (R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2] - 1.0)
    small = s2 < 1e-16
    s = torch.sqrt(torch.where(small, torch.ones_like(s2), s2))
    theta = torch.atan2(s, c)
    f = torch.where(small, 1.0 + s2 / 6.0, theta / s)   # theta / sin(theta)
    return f[..., None] * v


def log(R, t, s):
    """xi = (rho, phi, sigma) of (R, t, s) near the identity."""
    phi = so3_log(R)
    sigma = torch.log(s)
    rho = torch.linalg.solve(_w_matrix(phi, sigma), t[..., None])[..., 0]
    return torch.cat([rho, phi, sigma[..., None]], -1)


def compose(a, b):
    Ra, ta, sa = a
    Rb, tb, sb = b
    return Ra @ Rb, sa[..., None] * (Ra @ tb[..., None])[..., 0] + ta, sa * sb


def inverse(a):
    R, t, s = a
    Rt = R.transpose(-1, -2)
    return Rt, -(Rt @ t[..., None])[..., 0] / s[..., None], 1.0 / s


def from_poses(poses):
    """Similarities (R, t, 1) of camera-to-world poses [N, 7] (t, q)."""
    P = torch.as_tensor(np.asarray(poses, dtype=np.float64))
    return quat_to_rot(P[:, 3:]), P[:, :3].clone(), torch.ones(P.shape[0], dtype=F64)


def from_array(S):
    """(R, t, s) of similarities stored [N, 8] (t, q, s)."""
    S = torch.as_tensor(np.asarray(S, dtype=np.float64))
    return quat_to_rot(S[:, 3:7]), S[:, :3].clone(), S[:, 7].clone()


def to_array(S):
    R, t, s = (x.detach().numpy() for x in S)
    return np.concatenate([t, rot_to_quat(R), s[:, None]], 1)


def edge_list(n, loop_j, loop_k):
    """(a, b) of every residual: the N - 1 smoothness terms, then the loops."""
    a = np.concatenate([np.arange(n - 1), np.asarray(loop_j, dtype=np.int64)])
    b = np.concatenate([np.arange(1, n), np.asarray(loop_k, dtype=np.int64)])
    return a, b


def edge_constants(S0, loop_rel):
    """Per residual the constant C with r = log(C S_a^-1 S_b): DeltaS^-1 of
    consecutive initial similarities for eq. 5, DeltaS^loop for eq. 6."""
    R, t, s = S0
    D_odo = compose(inverse((R[:-1], t[:-1], s[:-1])), (R[1:], t[1:], s[1:]))
    Ci = inverse(D_odo)
    if loop_rel is None or len(loop_rel) == 0:
        return Ci
    Dl = from_array(loop_rel)
    return tuple(torch.cat([x, y], 0) for x, y in zip(Ci, Dl))


def residuals(S, C, a, b, da=None, db=None):
    """r_e = log(C_e (S_a Exp(da_e))^-1 (S_b Exp(db_e))) for every residual e."""
    R, t, s = S
    ia = torch.as_tensor(a)
    ib = torch.as_tensor(b)
    Sa = (R[ia], t[ia], s[ia])
    Sb = (R[ib], t[ib], s[ib])
    if da is not None:
        Sa = compose(Sa, exp(da))
        Sb = compose(Sb, exp(db))
    return log(*compose(C, compose(inverse(Sa), Sb)))


def cost(S, C, a, b):
    r = residuals(S, C, a, b)
    return float((r * r).sum())


def edge_jacobians(S, C, a, b):
    """r [E, 7] and the exact per-residual Jacobians d r_e / d delta_a,
    d r_e / d delta_b [E, 7, 7] (right perturbations), one reverse pass per
    residual component (each residual depends on its own two poses only)."""
    E = len(a)
    da = torch.zeros(E, 7, dtype=F64, requires_grad=True)
    db = torch.zeros(E, 7, dtype=F64, requires_grad=True)
    r = residuals(S, C, a, b, da, db)
    Ja = torch.zeros(E, 7, 7, dtype=F64)
    Jb = torch.zeros(E, 7, 7, dtype=F64)
    for c in range(7):
        ga, gb = torch.autograd.grad(r[:, c].sum(), (da, db), retain_graph=c < 6)
        Ja[:, c] = ga
        Jb[:, c] = gb
    return r.detach(), Ja, Jb


def retract(S, delta):
    """S_i Exp(delta_i) for every i (delta [N, 7])."""
    return compose(S, exp(delta))


def optimise(poses0, loop_j, loop_k, loop_rel, n_iters=10, lam=1e-4, n_fixed=1):
    """Similarities [N, 8] (t, q, s) after n_iters LM iterations of eq. 7, and
    the cost before each iteration and at the end."""
    S = from_poses(poses0)
    n = S[0].shape[0]
    a, b = edge_list(n, loop_j, loop_k)
    C = edge_constants(S, loop_rel)
    nf = n - n_fixed
    costs = []
    for _ in range(n_iters):
        r, Ja, Jb = edge_jacobians(S, C, a, b)
        costs.append(float((r * r).sum()))
        H = np.zeros((7 * n, 7 * n))
        g = np.zeros(7 * n)
        rn, Jan, Jbn = r.numpy(), Ja.numpy(), Jb.numpy()
        for e in range(len(a)):   # H = J^T J, g = J^T r, block by block in residual order
            for (p, Jp) in ((a[e], Jan[e]), (b[e], Jbn[e])):
                g[7 * p:7 * p + 7] += Jp.T @ rn[e]
                for (q, Jq) in ((a[e], Jan[e]), (b[e], Jbn[e])):
                    H[7 * p:7 * p + 7, 7 * q:7 * q + 7] += Jp.T @ Jq
        H = H[7 * n_fixed:, 7 * n_fixed:]
        g = g[7 * n_fixed:]
        Hd = H + lam * (np.diag(np.diag(H)) + np.eye(H.shape[0]))
        step = -np.linalg.solve(Hd, g)
        full = torch.cat([torch.zeros(n_fixed, 7, dtype=F64), torch.as_tensor(step.reshape(nf, 7))], 0)
        S = tuple(x.detach() for x in retract(S, full))
    costs.append(cost(S, C, a, b))
    return to_array(S), costs


def apply_to_ba(sims, poses, inv_depth, patch_owner):
    """G_i <- (t_i, R_i), d_k <- d_k / s_(owner(k)) (Sec. 3.3, last step)."""
    sims = np.asarray(sims, dtype=np.float64)
    P = np.asarray(poses, dtype=np.float64).copy()
    P[:, :3] = sims[:, :3]
    P[:, 3:] = sims[:, 3:7]
    d = np.asarray(inv_depth, dtype=np.float64) / sims[np.asarray(patch_owner), 7]
    return P, d
