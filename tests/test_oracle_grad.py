"""Pins for the gradient oracle (oracle/grad64.py): its forward agrees with
the independent numpy oracle, and its reverse-mode gradients with respect to
targets and weights agree with central finite differences of the loss."""
import numpy as np
import pytest
import torch

from oracle import ba64, grad64, lie64
from scenes import tiny_scene, make_config


def _same_rotation(pa, pb, atol):
    Ra, _ = lie64.pose_to_rt(pa)
    Rb, _ = lie64.pose_to_rt(pb)
    np.testing.assert_allclose(Ra, Rb, atol=atol)


@pytest.mark.parametrize("mk", [lambda: tiny_scene(5, 6, seed=31), lambda: tiny_scene(6, 5, seed=32, radius=2)])
def test_forward_matches_numpy_oracle(mk):
    s = mk()
    P, D, _ = ba64.solve_scene(s)
    poses, d = grad64.forward_state(s)
    np.testing.assert_allclose(poses[:, :3], P[:, :3], atol=1e-12)
    _same_rotation(poses, P, 1e-12)
    np.testing.assert_allclose(np.linalg.norm(poses[:, 3:], axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(d, D, rtol=1e-11)


def test_forward_matches_on_a_window():
    s = make_config(3, 0)
    P, D, _ = ba64.solve_scene(s)
    poses, d = grad64.forward_state(s)
    np.testing.assert_allclose(poses[:, :3], P[:, :3], atol=1e-11)
    _same_rotation(poses, P, 1e-11)
    np.testing.assert_allclose(d, D, rtol=1e-10)


def test_retraction_matches_se3_exp():
    """The (t, q) retraction equals G Exp(xi) with the closed-form SE(3) Exp."""
    rng = np.random.default_rng(5)
    for scale in (1e-4, 0.3, 2.0):
        t = rng.normal(size=(4, 3))
        q = rng.normal(size=(4, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        xi = rng.normal(size=(4, 6)) * scale
        tn, qn = grad64.retract_right(torch.as_tensor(t), torch.as_tensor(q), torch.as_tensor(xi))
        for a in range(4):
            G = np.eye(4)
            G[:3, :3] = lie64.quat_to_rot(q[a])
            G[:3, 3] = t[a]
            Re, te = lie64.se3_exp(xi[a])
            X = np.eye(4)
            X[:3, :3] = Re
            X[:3, 3] = te
            Gn = G @ X
            np.testing.assert_allclose(tn[a].numpy(), Gn[:3, 3], atol=1e-13)
            np.testing.assert_allclose(lie64.quat_to_rot(qn[a].numpy()), Gn[:3, :3], atol=1e-13)


@pytest.mark.parametrize("seed", [41, 42])
def test_gradients_match_central_differences(seed):
    s = tiny_scene(5, 5, seed=seed)
    L, gt, gw, _, _ = grad64.loss_and_grads(s)
    rng = np.random.default_rng(seed)
    h = 1e-6
    tgt = s.target.astype(np.float64)
    wgt = s.weight.astype(np.float64)
    for _ in range(12):
        e, c = int(rng.integers(s.n_edges)), int(rng.integers(2))
        for arr, g, name in ((tgt, gt, "target"), (wgt, gw, "weight")):
            ap, am = arr.copy(), arr.copy()
            ap[e, c] += h
            am[e, c] -= h
            if name == "target":
                fd = (grad64.loss_value(s, ap, wgt) - grad64.loss_value(s, am, wgt)) / (2 * h)
            else:
                fd = (grad64.loss_value(s, tgt, ap) - grad64.loss_value(s, tgt, am)) / (2 * h)
            assert abs(fd - g[e, c]) <= 1e-6 * max(1.0, abs(fd)) + 1e-5 * np.abs(g).max(), (name, e, c, fd, g[e, c])
    # a random direction over all coordinates
    dirs = rng.normal(size=tgt.shape)
    fd = (grad64.loss_value(s, tgt + h * dirs, wgt) - grad64.loss_value(s, tgt - h * dirs, wgt)) / (2 * h)
    assert abs(fd - np.sum(gt * dirs)) <= 1e-6 * max(1.0, abs(fd))


def test_gradients_with_held_poses_and_three_iterations():
    s = tiny_scene(6, 4, seed=43, n_fixed=2)
    L, gt, gw, _, _ = grad64.loss_and_grads(s, n_iters=3)
    rng = np.random.default_rng(43)
    h = 1e-6
    tgt = s.target.astype(np.float64)
    wgt = s.weight.astype(np.float64)
    for arr, g, which in ((tgt, gt, 0), (wgt, gw, 1)):
        dirs = rng.normal(size=arr.shape)
        if which == 0:
            fd = (grad64.loss_value(s, tgt + h * dirs, wgt, n_iters=3) -
                  grad64.loss_value(s, tgt - h * dirs, wgt, n_iters=3)) / (2 * h)
        else:
            fd = (grad64.loss_value(s, tgt, wgt + h * dirs, n_iters=3) -
                  grad64.loss_value(s, tgt, wgt - h * dirs, n_iters=3)) / (2 * h)
        assert abs(fd - np.sum(g * dirs)) <= 1e-6 * max(1.0, abs(fd))


def test_zero_iterations_give_zero_gradients():
    s = tiny_scene(4, 4, seed=44)
    L, gt, gw, gp, gd = grad64.loss_and_grads(s, n_iters=0)
    assert np.all(gt == 0) and np.all(gw == 0)
    assert np.abs(gp).max() > 0 and np.abs(gd).max() > 0


def test_pose_loss_closed_form():
    """Squared translation error plus squared rotation angle of R_ref^T R."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(7)
    ref = np.zeros((4, 7))
    ref[:, :3] = rng.normal(size=(4, 3))
    ref[:, 3:] = Rotation.from_rotvec(rng.normal(size=(4, 3))).as_quat()
    out = ref.copy()
    want = 0.0
    for a in range(2, 4):  # poses 0, 1 held: excluded from the loss
        delta = rng.normal(size=3) * 0.3
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        theta = 0.05 + 0.4 * a
        out[a, :3] += delta
        R = Rotation.from_quat(ref[a, 3:]) * Rotation.from_rotvec(theta * axis)
        q = R.as_quat()
        out[a, 3:] = -q if a == 3 else q  # the sign of a quaternion does not matter
        want += float(delta @ delta) + theta ** 2
    out[0, :3] += 5.0  # held pose: ignored
    L = grad64.pose_loss(torch.as_tensor(out), torch.as_tensor(ref), 2)
    assert abs(float(L) - want) < 1e-12 * max(1.0, want)


def test_rotation_angle_gradient_finite_at_zero():
    q = torch.tensor([[0.1, -0.2, 0.3, 0.9]], dtype=torch.float64)
    q = (q / q.norm()).requires_grad_(True)
    a2 = grad64.rotation_angle_sq(q, q.detach().clone())
    (g,) = torch.autograd.grad(a2.sum(), q)
    assert float(a2) < 1e-30 and torch.isfinite(g).all() and float(g.abs().max()) < 1e-12
    # small angle: derivative of theta^2 along the generator matches central differences
    from scipy.spatial.transform import Rotation
    base = Rotation.from_rotvec([0.0, 0.0, 1e-3])
    qq = torch.as_tensor(base.as_quat()[None], dtype=torch.float64)
    ref = torch.tensor([[0.0, 0.0, 0.0, 1.0]], dtype=torch.float64)
    assert abs(float(grad64.rotation_angle_sq(qq, ref)) - 1e-6) < 1e-18


def test_pose_loss_gradients_match_central_differences():
    s = tiny_scene(5, 5, seed=49)
    loss = grad64.scene_pose_loss(s)
    L, gt, gw, _, _ = grad64.loss_and_grads(s, loss_fn=loss)
    rng = np.random.default_rng(49)
    h = 1e-6
    tgt = s.target.astype(np.float64)
    wgt = s.weight.astype(np.float64)
    for arr, g, which in ((tgt, gt, 0), (wgt, gw, 1)):
        dirs = rng.normal(size=arr.shape)
        if which == 0:
            fd = (grad64.loss_value(s, tgt + h * dirs, wgt, loss_fn=loss) -
                  grad64.loss_value(s, tgt - h * dirs, wgt, loss_fn=loss)) / (2 * h)
        else:
            fd = (grad64.loss_value(s, tgt, wgt + h * dirs, loss_fn=loss) -
                  grad64.loss_value(s, tgt, wgt - h * dirs, loss_fn=loss)) / (2 * h)
        assert abs(fd - np.sum(g * dirs)) <= 1e-6 * max(1.0, abs(fd)), (which, fd, np.sum(g * dirs))


def test_levenberg_forward_and_gradients():
    """With the plain H + lam I damping the gradient oracle still agrees with
    the numpy oracle's forward and with central differences."""
    s = tiny_scene(5, 5, seed=50)
    s.lam = 1e-2
    P, D, _ = ba64.solve_scene(s, levenberg=True)
    poses, d = grad64.forward_state(s, levenberg=True)
    np.testing.assert_allclose(poses[:, :3], P[:, :3], atol=1e-12)
    np.testing.assert_allclose(d, D, rtol=1e-11)
    L, gt, gw, _, _ = grad64.loss_and_grads(s, levenberg=True)
    rng = np.random.default_rng(50)
    h = 1e-6
    tgt = s.target.astype(np.float64)
    wgt = s.weight.astype(np.float64)
    dirs = rng.normal(size=wgt.shape)
    fd = (grad64.loss_value(s, tgt, wgt + h * dirs, levenberg=True) -
          grad64.loss_value(s, tgt, wgt - h * dirs, levenberg=True)) / (2 * h)
    assert abs(fd - np.sum(gw * dirs)) <= 1e-6 * max(1.0, abs(fd))
