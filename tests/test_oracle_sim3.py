"""Pins of the Sim(3) pose-graph oracle (oracle/sim3_pgo.py, eq. 5-7):
Exp against scipy's matrix exponential of the 4x4 similarity generator, Log
as its inverse, composition and inverse as 4x4 matrix products, autograd
Jacobians against central differences, the fixed point of consistent
measurements, stationarity after convergence, gauge covariance, and the
pose / depth update."""
import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import sim3_pgo as P

F64 = torch.float64


def _mat4(R, t, s):
    M = np.eye(4)
    M[:3, :3] = float(s) * np.asarray(R)
    M[:3, 3] = np.asarray(t)
    return M


def _gen4(xi):
    rho, phi, sigma = xi[:3], xi[3:6], xi[6]
    G = np.zeros((4, 4))
    G[:3, :3] = sigma * np.eye(3) + np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    G[:3, 3] = rho
    return G


@pytest.mark.parametrize("seed", range(5))
def test_exp_is_the_matrix_exponential_and_log_inverts_it(seed):
    rng = np.random.default_rng(seed)
    xi = rng.normal(size=7) * np.array([1, 1, 1, 0.8, 0.8, 0.8, 0.5])
    R, t, s = P.exp(torch.as_tensor(xi[None]))
    got = _mat4(R[0].numpy(), t[0].numpy(), s[0].item())
    want = scipy.linalg.expm(_gen4(xi))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    back = P.log(R, t, s)[0].numpy()
    np.testing.assert_allclose(back, xi, rtol=1e-10, atol=1e-12)
    # tiny arguments take the series branch of the rotation log
    xi_s = xi * 1e-9
    np.testing.assert_allclose(P.log(*P.exp(torch.as_tensor(xi_s[None])))[0].numpy(), xi_s, rtol=1e-6, atol=1e-20)


def test_compose_and_inverse_are_matrix_products():
    rng = np.random.default_rng(3)
    a = P.exp(torch.as_tensor(rng.normal(size=(1, 7))))
    b = P.exp(torch.as_tensor(rng.normal(size=(1, 7))))
    Ma = _mat4(a[0][0].numpy(), a[1][0].numpy(), a[2][0].item())
    Mb = _mat4(b[0][0].numpy(), b[1][0].numpy(), b[2][0].item())
    c = P.compose(a, b)
    np.testing.assert_allclose(_mat4(c[0][0].numpy(), c[1][0].numpy(), c[2][0].item()), Ma @ Mb, rtol=1e-12,
                               atol=1e-12)
    ia = P.inverse(a)
    np.testing.assert_allclose(_mat4(ia[0][0].numpy(), ia[1][0].numpy(), ia[2][0].item()), np.linalg.inv(Ma),
                               rtol=1e-12, atol=1e-12)


def _problem(n=40, seed=0, drift=0.05, loops=((2, 30), (5, 36), (10, 38))):
    """A planar loop: ground truth on a circle, the estimate with scale and
    heading drift; loop measurements from the ground truth."""
    rng = np.random.default_rng(seed)
    ang = np.linspace(0, 2 * np.pi * 0.95, n)
    c_gt = np.stack([5 * np.cos(ang), 5 * np.sin(ang), 0.1 * rng.normal(size=n)], 1)
    from scipy.spatial.transform import Rotation
    R_gt = Rotation.from_euler("z", ang + np.pi / 2).as_matrix()
    steps = np.diff(c_gt, axis=0) * (1 + drift * np.arange(1, n)[:, None] / n)
    c0 = np.concatenate([c_gt[:1], c_gt[0] + np.cumsum(steps, 0)], 0)
    R0 = Rotation.from_euler("z", ang + np.pi / 2 + 0.02 * np.arange(n) / n).as_matrix()
    pose = lambda R, c: np.concatenate([c, P.rot_to_quat(R)], 1)
    poses0, poses_gt = pose(R0, c0), pose(R_gt, c_gt)
    gt = P.from_poses(poses_gt)
    lj = [a for a, _ in loops]
    lk = [b for _, b in loops]
    D = P.compose(P.inverse((gt[0][lj], gt[1][lj], gt[2][lj])), (gt[0][lk], gt[1][lk], gt[2][lk]))
    loop_rel = P.to_array(P.inverse(D))   # the loop residual vanishes at ground truth
    return poses0, poses_gt, lj, lk, loop_rel


def test_jacobians_match_central_differences():
    poses0, _, lj, lk, loop_rel = _problem(12, loops=((1, 9), (2, 11)))
    S = P.from_poses(poses0)
    # a non-trivial point: move the similarities away from the start
    rng = np.random.default_rng(1)
    S = P.retract(S, torch.as_tensor(0.05 * rng.normal(size=(12, 7))))
    a, b = P.edge_list(12, lj, lk)
    C = P.edge_constants(P.from_poses(poses0), loop_rel)
    r, Ja, Jb = P.edge_jacobians(S, C, a, b)
    h = 1e-6
    for side, J in ((0, Ja), (1, Jb)):
        for d in range(7):
            e = torch.zeros(len(a), 7, dtype=F64)
            e[:, d] = h
            z = torch.zeros(len(a), 7, dtype=F64)
            args_p = (e, z) if side == 0 else (z, e)
            args_m = (-e, z) if side == 0 else (z, -e)
            fd = (P.residuals(S, C, a, b, *args_p) - P.residuals(S, C, a, b, *args_m)) / (2 * h)
            np.testing.assert_allclose(J[:, :, d].numpy(), fd.numpy(), rtol=1e-6, atol=1e-8)


def test_consistent_measurements_are_a_fixed_point():
    _, poses_gt, lj, lk, loop_rel = _problem()
    sims, costs = P.optimise(poses_gt, lj, lk, loop_rel, n_iters=3)
    assert max(costs) < 1e-20
    np.testing.assert_allclose(sims[:, :3], poses_gt[:, :3], atol=1e-12)
    np.testing.assert_allclose(sims[:, 7], 1.0, atol=1e-12)


def test_drift_is_corrected_to_a_stationary_point():
    poses0, poses_gt, lj, lk, loop_rel = _problem()
    sims, costs = P.optimise(poses0, lj, lk, loop_rel, n_iters=25, lam=1e-6)
    assert costs[-1] < 1e-2 * costs[0]   # odometry drift and loops cannot all be met: a compromise remains
    S = P.from_array(sims)
    a, b = P.edge_list(len(poses0), lj, lk)
    C = P.edge_constants(P.from_poses(poses0), loop_rel)
    r, Ja, Jb = P.edge_jacobians(S, C, a, b)
    g = np.zeros((len(poses0), 7))
    np.add.at(g, a, np.einsum("eij,ei->ej", Ja.numpy(), r.numpy()))
    np.add.at(g, b, np.einsum("eij,ei->ej", Jb.numpy(), r.numpy()))
    assert np.abs(g[1:]).max() < 1e-9 * max(1.0, costs[0])
    # the corrected end is closer to the truth than the drifted start
    err0 = np.linalg.norm(poses0[:, :3] - poses_gt[:, :3], axis=1).max()
    err1 = np.linalg.norm(sims[:, :3] - poses_gt[:, :3], axis=1).max()
    assert err1 < err0


def test_gauge_covariance():
    """A rigid transform T applied to every starting pose moves the result by T."""
    poses0, _, lj, lk, loop_rel = _problem(20, loops=((1, 15), (3, 18)))
    sims, _ = P.optimise(poses0, lj, lk, loop_rel, n_iters=4)
    from scipy.spatial.transform import Rotation
    Rt = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    tt = np.array([1.0, -2.0, 0.5])
    S0 = P.from_poses(poses0)
    R1 = np.einsum("ab,nbc->nac", Rt, S0[0].numpy())
    c1 = S0[1].numpy() @ Rt.T + tt
    poses1 = np.concatenate([c1, P.rot_to_quat(R1)], 1)
    sims1, _ = P.optimise(poses1, lj, lk, loop_rel, n_iters=4)
    np.testing.assert_allclose(sims1[:, :3], sims[:, :3] @ Rt.T + tt, atol=1e-9)
    np.testing.assert_allclose(sims1[:, 7], sims[:, 7], atol=1e-12)


def test_apply_to_ba():
    sims = np.array([[1.0, 2.0, 3.0, 0.0, 0.0, 0.0, 1.0, 2.0], [0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.5]])
    P_, d = P.apply_to_ba(sims, np.zeros((2, 7)), np.array([1.0, 2.0, 3.0]), np.array([0, 0, 1]))
    np.testing.assert_allclose(P_, sims[:, :7])
    np.testing.assert_allclose(d, [0.5, 1.0, 6.0])
