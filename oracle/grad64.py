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

The iterate is carried in the stored coordinates (t, q) of the poses, so
the gradients with respect to the final poses are the ones a caller
computes on the returned [N,7] array.
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


def quat_mul(a, b):
    """Hamilton product of (x, y, z, w) quaternions."""
    ax, ay, az, aw = a.unbind(-1)
    bx, by, bz, bw = b.unbind(-1)
    return torch.stack([aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw,
                        aw * bw - ax * bx - ay * by - az * bz], -1)


def retract_right(t, q, xi):
    """G Exp(xi) on the stored coordinates: t + R V(phi) rho and the
    normalised q (x) (sin(theta/2) phi / theta, cos(theta/2))."""
    rho, phi = xi[..., :3], xi[..., 3:]
    A, B, C = _exp_coeffs(phi)
    th2 = (phi * phi).sum(-1)
    small = th2 < 1e-4
    th = torch.where(small, torch.ones_like(th2), th2).sqrt()
    h = torch.where(small, 0.5 - th2 / 48 + th2 * th2 / 3840, torch.sin(th / 2) / th)
    ch = torch.where(small, 1 - th2 / 8 + th2 * th2 / 384, torch.cos(th / 2))
    K = _hat(phi)
    I = torch.eye(3, dtype=DT).expand(K.shape)
    V = I + B[..., None, None] * K + C[..., None, None] * (K @ K)
    R = quat_to_rot(q)
    tn = t + (R @ (V @ rho[..., None]))[..., 0]
    qn = quat_mul(q, torch.cat([h[..., None] * phi, ch[..., None]], -1))
    return tn, qn / qn.norm(dim=-1, keepdim=True)


def gn_iteration(t, q, d, centres, ii, jj, kk, target, weight, intr, n_fixed, lam, z_min, levenberg=False):
    """One damped GN step on the stored coordinates; returns (t, q, d).
    Damping H + lam (Diag(H) + I), or H + lam I with levenberg=True."""
    fx, fy, cx, cy = intr
    R = quat_to_rot(q)
    N, P = R.shape[0], d.shape[0]
    Rj_T = R[jj].transpose(-1, -2)
    Rji = Rj_T @ R[ii]
    tji = (Rj_T @ (t[ii] - t[jj])[..., None])[..., 0]
    xh = torch.stack([(centres[kk, 0] - cx) / fx, (centres[kk, 1] - cy) / fy,
                      torch.ones(kk.shape[0], dtype=DT)], -1)
    dk = d[kk]
    pt = (Rji @ xh[..., None])[..., 0] + tji * dk[:, None]
    valid = ((dk > 0) & (pt[:, 2] > z_min * dk)).to(DT)
    z = torch.where(valid > 0, pt[:, 2], torch.ones_like(pt[:, 2]))
    r = torch.stack([fx * pt[:, 0] / z + cx, fy * pt[:, 1] / z + cy], -1) - target
    E = pt.shape[0]
    zero = torch.zeros(E, dtype=DT)
    Jpi = torch.stack([torch.stack([fx / z, zero, -fx * pt[:, 0] / (z * z)], -1),
                       torch.stack([zero, fy / z, -fy * pt[:, 1] / (z * z)], -1)], -2)
    eye = torch.eye(3, dtype=DT).expand(E, 3, 3)
    Jj = Jpi @ torch.cat([-dk[:, None, None] * eye, _hat(pt)], -1)
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
    mq = 0.0 if levenberg else 1.0
    Bt = B + lam * torch.diag(mq * torch.diagonal(B) + 1)
    Ct = C + lam * (mq * C + 1)
    S = Bt - (Em / Ct) @ Em.T
    s = -v + Em @ (gd / Ct)
    if n:
        L = torch.linalg.cholesky(S)
        dxi = torch.cholesky_solve(s[:, None], L)[:, 0]
    else:
        dxi = torch.zeros(0, dtype=DT)
    dd = (-gd - Em.T @ dxi) / Ct
    tn, qn = retract_right(t[nf:], q[nf:], dxi.reshape(Nf, 6))
    return torch.cat([t[:nf], tn], 0), torch.cat([q[:nf], qn], 0), d + dd


def unrolled(poses0, d0, centres, ii, jj, kk, target, weight, intr, n_fixed, n_iters, lam, z_min, levenberg=False):
    """poses [N,7] (t, q) and depths [P] after n_iters iterations."""
    t, q, d = poses0[:, :3], poses0[:, 3:], d0
    for _ in range(n_iters):
        t, q, d = gn_iteration(t, q, d, centres, ii, jj, kk, target, weight, intr, n_fixed, lam, z_min, levenberg)
    return torch.cat([t, q], -1), d


def rotation_angle_sq(q, q_ref):
    """||Log(R_ref^T R)||^2 of unit quaternions (x, y, z, w): the squared angle
    2 atan2(|v|, |w|) of the relative rotation q_ref^-1 q = (v, w), written so
    that autograd stays finite at zero angle (atan2(s, c) / s -> 1 / c)."""
    qr_inv = torch.cat([-q_ref[..., :3], q_ref[..., 3:]], -1)
    rel = quat_mul(qr_inv, q / q.norm(dim=-1, keepdim=True))
    v, w = rel[..., :3], rel[..., 3].abs()
    s2 = (v * v).sum(-1)
    small = s2 < 1e-24
    s = torch.where(small, torch.ones_like(s2), s2).sqrt()
    f = torch.where(small, 1.0 / w, torch.atan2(s, w) / s)
    return 4.0 * f * f * s2


def pose_loss(poses, poses_ref, n_fixed):
    """The supervision loss on the poses BA produces (the differentiable BA
    layer of Sec. 2): sum over free poses of ||t - t_ref||^2 + ||Log(R_ref^T R)||^2."""
    t, q = poses[n_fixed:, :3], poses[n_fixed:, 3:]
    tr, qr = poses_ref[n_fixed:, :3], poses_ref[n_fixed:, 3:]
    return ((t - tr) ** 2).sum() + rotation_angle_sq(q, qr).sum()


def scene_pose_loss(scene):
    """pose_loss against the scene's ground-truth poses, as a callable of (poses, d)."""
    ref = torch.as_tensor(scene.poses_gt, dtype=DT)
    return lambda poses, d: pose_loss(poses, ref, int(scene.n_fixed))


def pose_depth_loss(poses, d, poses_ref, d_ref, n_fixed):
    """A test loss touching every output: squared translation error,
    1 - <q, q_ref>^2 per free pose (sign invariant), and the mean squared
    inverse-depth error."""
    t, q = poses[n_fixed:, :3], poses[n_fixed:, 3:]
    tr, qr = poses_ref[n_fixed:, :3], poses_ref[n_fixed:, 3:]
    return ((t - tr) ** 2).sum() + (1 - (q * qr).sum(-1) ** 2).sum() + ((d - d_ref) ** 2).mean()


def scene_loss(scene):
    """pose_depth_loss against the scene's ground truth, as a callable."""
    ref = torch.as_tensor(scene.poses_gt, dtype=DT)
    dref = torch.as_tensor(scene.inv_depth_gt, dtype=DT)
    return lambda poses, d: pose_depth_loss(poses, d, ref, dref, int(scene.n_fixed))


def _tensors(scene):
    c = (scene.patches.shape[1] - 1) // 2
    return dict(
        poses0=torch.as_tensor(scene.poses, dtype=DT), d0=torch.as_tensor(scene.inv_depth, dtype=DT),
        centres=torch.as_tensor(scene.patches[:, c, c, :], dtype=DT),
        ii=torch.as_tensor(scene.ii, dtype=torch.long), jj=torch.as_tensor(scene.jj, dtype=torch.long),
        kk=torch.as_tensor(scene.kk, dtype=torch.long), intr=[float(x) for x in scene.intrinsics],
        n_fixed=int(scene.n_fixed))


def _run(scene, target, weight, n_iters, lam, z_min, track=False, levenberg=False):
    T = _tensors(scene)
    if track:  # keep the outputs in the graph even without iterations
        T["poses0"].requires_grad_(True)
        T["d0"].requires_grad_(True)
    return unrolled(T["poses0"], T["d0"], T["centres"], T["ii"], T["jj"], T["kk"], target, weight, T["intr"],
                    T["n_fixed"], scene.n_iters if n_iters is None else n_iters,
                    scene.lam if lam is None else lam, scene.z_min if z_min is None else z_min, levenberg)


def loss_and_grads(scene, loss_fn=None, n_iters=None, lam=None, z_min=None, levenberg=False):
    """L = loss_fn(poses_T, d_T) after the unrolled iterations, and (numpy
    float64) dL/d target [E,2], dL/d weight [E,2], dL/d poses_T [N,7],
    dL/d d_T [P].  loss_fn defaults to scene_loss(scene)."""
    loss_fn = scene_loss(scene) if loss_fn is None else loss_fn
    target = torch.as_tensor(scene.target, dtype=DT).clone().requires_grad_(True)
    weight = torch.as_tensor(scene.weight, dtype=DT).clone().requires_grad_(True)
    poses, d = _run(scene, target, weight, n_iters, lam, z_min, track=True, levenberg=levenberg)
    L = loss_fn(poses, d)
    ins = (target, weight, poses, d)
    gr = torch.autograd.grad(L, ins, allow_unused=True)
    gt, gw, gp, gd = (torch.zeros_like(x) if g is None else g for g, x in zip(gr, ins))
    return float(L.detach()), gt.numpy(), gw.numpy(), gp.detach().numpy(), gd.detach().numpy()


def loss_value(scene, target, weight, loss_fn=None, n_iters=None, lam=None, z_min=None, levenberg=False):
    """The loss alone, for given float64 targets / weights (numpy)."""
    loss_fn = scene_loss(scene) if loss_fn is None else loss_fn
    with torch.no_grad():
        poses, d = _run(scene, torch.as_tensor(target, dtype=DT), torch.as_tensor(weight, dtype=DT), n_iters,
                        lam, z_min, levenberg=levenberg)
        return float(loss_fn(poses, d))


def forward_state(scene, n_iters=None, levenberg=False):
    """(poses [N,7], d [P]) after the unrolled iterations, numpy float64."""
    with torch.no_grad():
        poses, d = _run(scene, torch.as_tensor(scene.target, dtype=DT), torch.as_tensor(scene.weight, dtype=DT),
                        n_iters, None, None, levenberg=levenberg)
    return poses.numpy(), d.numpy()
