"""Gradient oracle: float64 reverse-mode derivatives of the unrolled
Gauss-Newton iterations (test infrastructure only; see the package docstring).

The differentiable BA layer of DPVO/DPV-SLAM (Sec. 2: supervision on the
predicted camera poses through bundle adjustment) needs dL/d(target) and
dL/d(weight) for a loss on the poses after a fixed number of GN iterations.
This module states the same iteration as `ba64` -- eq. 2 reprojection, eq. 3
normal equations with the Marquardt damping H + lam (Diag(H) + I), Schur
elimination of the depths, Cholesky solve, right SE(3) retraction -- in
torch float64 with dense blocks, so that autograd differentiates through
every step, including the Jacobians' dependence on the iterate and the
factorisation.  It is written independently of `ba64` (torch tensors,
dense block assembly by index_add) so that the two cross-check each other.

Loss (pose L2 error): L = sum over free poses of |t_i - t_i^gt|^2 +
|Log(R_i^gt^T R_i)|^2.
"""
from __future__ import annotations

import torch

DT = torch.float64


def _hat(v):
    z = torch.zeros_like(v[..., 0])
    return torch.stack([torch.stack([z, -v[..., 2], v[..., 1]], -1),
                        torch.stack([v[..., 2], z, -v[..., 0]], -1),
                        torch.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def quat_to_rot(q):
    q = q / q.norm(dim=-1, keepdim=True)
    x, y, z, w = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], -2)


def _exp_coeffs(phi):
    """sin(t)/t, (1 - cos t)/t^2, (t - sin t)/t^3 with a series below t^2 = 1e-4
    (branch values are finite on both sides so autograd stays finite)."""
    th2 = (phi * phi).sum(-1)
    small = th2 < 1e-4
    th2s = torch.where(small, torch.ones_like(th2), th2)
    th = th2s.sqrt()
    A = torch.where(small, 1 - th2 / 6 + th2 * th2 / 120, torch.sin(th) / th)
    B = torch.where(small, 0.5 - th2 / 24 + th2 * th2 / 720, (1 - torch.cos(th)) / th2s)
    C = torch.where(small, 1.0 / 6 - th2 / 120 + th2 * th2 / 5040, (th - torch.sin(th)) / (th2s * th))
    return A, B, C


def retract_right(R, t, xi):
    """G Exp(xi): R Exp(phi), t + R V(phi) rho."""
    rho, phi = xi[..., :3], xi[..., 3:]
    A, B, C = _exp_coeffs(phi)
    K = _hat(phi)
    I = torch.eye(3, dtype=DT).expand(K.shape)
    K2 = K @ K
    dR = I + A[..., None, None] * K + B[..., None, None] * K2
    V = I + B[..., None, None] * K + C[..., None, None] * K2
    return R @ dR, t + (R @ (V @ rho[..., None]))[..., 0]


def rot_log_sq(R):
    """|Log(R)|^2 via the rotation angle theta = atan2(|v|, (tr R - 1) / 2)."""
    v = torch.stack([R[..., 2, 1] - R[..., 1, 2], R[..., 0, 2] - R[..., 2, 0], R[..., 1, 0] - R[..., 0, 1]], -1) / 2
    c = (R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2] - 1) / 2
    s = v.norm(dim=-1)
    return torch.atan2(s, c) ** 2


def gn_iteration(R, t, d, centres, ii, jj, kk, target, weight, intr, n_fixed, lam, z_min):
    """One damped GN step; returns the updated (R, t, d)."""
    fx, fy, cx, cy = intr
    N, P = R.shape[0], d.shape[0]
    Rj_T = R[jj].transpose(-1, -2)
    Rji = Rj_T @ R[ii]
    tji = (Rj_T @ (t[ii] - t[jj])[..., None])[..., 0]
    xh = torch.stack([(centres[kk, 0] - cx) / fx, (centres[kk, 1] - cy) / fy,
                      torch.ones(kk.shape[0], dtype=DT)], -1)
    dk = d[kk]
    q = (Rji @ xh[..., None])[..., 0] + tji * dk[:, None]
    valid = ((dk > 0) & (q[:, 2] > z_min * dk)).to(DT)
    z = torch.where(valid > 0, q[:, 2], torch.ones_like(q[:, 2]))
    r = torch.stack([fx * q[:, 0] / z + cx, fy * q[:, 1] / z + cy], -1) - target
    E = q.shape[0]
    zero = torch.zeros(E, dtype=DT)
    Jpi = torch.stack([torch.stack([fx / z, zero, -fx * q[:, 0] / (z * z)], -1),
                       torch.stack([zero, fy / z, -fy * q[:, 1] / (z * z)], -1)], -2)
    eye = torch.eye(3, dtype=DT).expand(E, 3, 3)
    Jj = Jpi @ torch.cat([-dk[:, None, None] * eye, _hat(q)], -1)
    Ji = Jpi @ Rji @ torch.cat([dk[:, None, None] * eye, -_hat(xh)], -1)
    Jd = (Jpi @ tji[..., None])[..., 0]
    W = weight * valid[:, None]
    # dense block assembly over the free poses (index nf..N-1 -> 0..N'-1)
    nf = n_fixed
    Nf = N - nf
    n = 6 * Nf
    Bpp = torch.zeros(Nf * Nf, 6, 6, dtype=DT)
    Epd = torch.zeros(Nf * P, 6, dtype=DT)
    C = torch.zeros(P, dtype=DT)
    gp = torch.zeros(Nf, 6, dtype=DT)
    gd = torch.zeros(P, dtype=DT)
    WJi = W[..., None] * Ji
    WJj = W[..., None] * Jj
    Wr = W * r
    WJd = W * Jd
    fi = ii >= nf
    fj = jj >= nf
    a, b = ii - nf, jj - nf
    for sel, x, y, X, Y in ((fi, a, a, Ji, WJi), (fj, b, b, Jj, WJj), (fi & fj, a, b, Ji, WJj),
                            (fi & fj, b, a, Jj, WJi)):
        blocks = X[sel].transpose(-1, -2) @ Y[sel]
        Bpp = Bpp.index_add(0, (x[sel] * Nf + y[sel]), blocks)
    for sel, x, X in ((fi, a, Ji), (fj, b, Jj)):
        Epd = Epd.index_add(0, x[sel] * P + kk[sel], (X[sel].transpose(-1, -2) @ WJd[sel][..., None])[..., 0])
        gp = gp.index_add(0, x[sel], (X[sel].transpose(-1, -2) @ Wr[sel][..., None])[..., 0])
    C = C.index_add(0, kk, (Jd * WJd).sum(-1))
    gd = gd.index_add(0, kk, (Jd * Wr).sum(-1))
    B = Bpp.reshape(Nf, Nf, 6, 6).permute(0, 2, 1, 3).reshape(n, n)
    Em = Epd.reshape(Nf, P, 6).permute(0, 2, 1).reshape(n, P)
    v = gp.reshape(n)
    Bt = B + lam * torch.diag(torch.diagonal(B) + 1)
    Ct = C + lam * (C + 1)
    S = Bt - (Em / Ct) @ Em.T
    s = -v + Em @ (gd / Ct)
    if n:
        L = torch.linalg.cholesky(S)
        dxi = torch.cholesky_solve(s[:, None], L)[:, 0]
    else:
        dxi = torch.zeros(0, dtype=DT)
    dd = (-gd - Em.T @ dxi) / Ct
    Rn, tn = retract_right(R[nf:], t[nf:], dxi.reshape(Nf, 6))
    return torch.cat([R[:nf], Rn], 0), torch.cat([t[:nf], tn], 0), d + dd


def unrolled(poses0, d0, centres, ii, jj, kk, target, weight, intr, n_fixed, n_iters, lam, z_min):
    R, t = quat_to_rot(poses0[:, 3:]), poses0[:, :3]
    d = d0
    for _ in range(n_iters):
        R, t, d = gn_iteration(R, t, d, centres, ii, jj, kk, target, weight, intr, n_fixed, lam, z_min)
    return R, t, d


def pose_loss(R, t, poses_gt, n_fixed):
    Rg, tg = quat_to_rot(poses_gt[:, 3:]), poses_gt[:, :3]
    Rr = Rg[n_fixed:].transpose(-1, -2) @ R[n_fixed:]
    return ((t[n_fixed:] - tg[n_fixed:]) ** 2).sum() + rot_log_sq(Rr).sum()


def _tensors(scene):
    c = (scene.patches.shape[1] - 1) // 2
    return dict(
        poses0=torch.as_tensor(scene.poses, dtype=DT), d0=torch.as_tensor(scene.inv_depth, dtype=DT),
        centres=torch.as_tensor(scene.patches[:, c, c, :], dtype=DT),
        ii=torch.as_tensor(scene.ii, dtype=torch.long), jj=torch.as_tensor(scene.jj, dtype=torch.long),
        kk=torch.as_tensor(scene.kk, dtype=torch.long), intr=[float(x) for x in scene.intrinsics],
        n_fixed=int(scene.n_fixed), poses_gt=torch.as_tensor(scene.poses_gt, dtype=DT))


def loss_and_grads(scene, n_iters=None, lam=None, z_min=None):
    """Loss after the unrolled iterations and its gradients with respect to
    the targets [E,2] and weights [E,2] (numpy float64)."""
    T = _tensors(scene)
    target = torch.as_tensor(scene.target, dtype=DT).clone().requires_grad_(True)
    weight = torch.as_tensor(scene.weight, dtype=DT).clone().requires_grad_(True)
    R, t, d = unrolled(T["poses0"], T["d0"], T["centres"], T["ii"], T["jj"], T["kk"], target, weight, T["intr"],
                       T["n_fixed"], scene.n_iters if n_iters is None else n_iters,
                       scene.lam if lam is None else lam, scene.z_min if z_min is None else z_min)
    L = pose_loss(R, t, T["poses_gt"], T["n_fixed"])
    gt, gw = torch.autograd.grad(L, (target, weight))
    return float(L.detach()), gt.numpy(), gw.numpy()


def loss_value(scene, target, weight, n_iters=None, lam=None, z_min=None):
    """The loss alone, for given float64 targets / weights (numpy)."""
    T = _tensors(scene)
    with torch.no_grad():
        R, t, d = unrolled(T["poses0"], T["d0"], T["centres"], T["ii"], T["jj"], T["kk"],
                           torch.as_tensor(target, dtype=DT), torch.as_tensor(weight, dtype=DT), T["intr"],
                           T["n_fixed"], scene.n_iters if n_iters is None else n_iters,
                           scene.lam if lam is None else lam, scene.z_min if z_min is None else z_min)
        return float(pose_loss(R, t, T["poses_gt"], T["n_fixed"]))


def forward_state(scene, n_iters=None):
    """(R [N,3,3], t [N,3], d [P]) after the unrolled iterations, numpy float64."""
    T = _tensors(scene)
    with torch.no_grad():
        R, t, d = unrolled(T["poses0"], T["d0"], T["centres"], T["ii"], T["jj"], T["kk"],
                           torch.as_tensor(scene.target, dtype=DT), torch.as_tensor(scene.weight, dtype=DT),
                           T["intr"], T["n_fixed"], scene.n_iters if n_iters is None else n_iters, scene.lam,
                           scene.z_min)
    return R.numpy(), t.numpy(), d.numpy()
