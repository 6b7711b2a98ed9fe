"""Pins for the float64 oracle of patch-graph Gauss-Newton BA.

Each test pins the oracle to something other than itself: closed forms of the
pinhole transfer (eq. 2), central finite differences, a dense solve of the
full damped normal equations built from a finite-difference Jacobian, the
large-damping limit, and invariants of the objective (eq. 3): the ground
truth as a fixed point, recovery of the ground truth, rigid-gauge
equivariance, monocular scale invariance, edge-order invariance and
duplicated-edge = doubled-weight.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import ba64, lie64
from scenes import tiny_scene, make_config


def _problem_single_edge(u, v, d, pose_i, pose_j, fx=320.0, fy=320.0, cx=320.0, cy=240.0):
    return ba64.Problem(
        poses=np.stack([pose_i, pose_j]).astype(np.float64),
        centres=np.array([[u, v]], dtype=np.float64), inv_depth=np.array([d]),
        ii=np.array([0]), jj=np.array([1]), kk=np.array([0]),
        target=np.zeros((1, 2)), weight=np.ones((1, 2)),
        intrinsics=np.array([fx, fy, cx, cy]), n_fixed=0,
        patches=np.array([[[[u + b - 1, v + a - 1] for b in range(3)] for a in range(3)]], dtype=np.float64))


IDENT = np.array([0, 0, 0, 0, 0, 0, 1.0])


def _pose(t, rotvec=(0, 0, 0)):
    return np.concatenate([np.asarray(t, float), Rotation.from_rotvec(rotvec).as_quat()])


# ---------------------------------------------------------------- closed forms

def test_identity_relative_pose_reprojects_to_same_pixel():
    pb = _problem_single_edge(400.0, 123.0, 0.5, IDENT, IDENT)
    t = ba64.edge_terms(pb)
    np.testing.assert_allclose(t.proj, [[400.0, 123.0]], atol=1e-12)
    full, valid = ba64.reproject(pb)
    np.testing.assert_allclose(full[0], pb.patches[0], atol=1e-12)
    assert valid.all()


def test_sideways_translation_closed_form():
    # camera j displaced by (b, 0, 0): u' = u - fx b d (paper eq. 2, worked by hand)
    pb = _problem_single_edge(400.0, 200.0, 0.5, IDENT, _pose([0.1, 0, 0]))
    t = ba64.edge_terms(pb)
    np.testing.assert_allclose(t.proj[0], [384.0, 200.0], atol=1e-12)


def test_forward_translation_closed_form():
    # camera j displaced by (0, 0, b): u' = cx + (u - cx) / (1 - b d)
    pb = _problem_single_edge(400.0, 240.0, 0.5, IDENT, _pose([0, 0, 0.1]))
    t = ba64.edge_terms(pb)
    np.testing.assert_allclose(t.proj[0], [320.0 + 80.0 / 0.95, 240.0], atol=1e-12)
    np.testing.assert_allclose(t.proj[0, 0], 404.2105263157895, atol=1e-12)


def test_pure_rotation_is_depth_independent():
    # a rotation-only relative pose maps pixels by the homography K R K^-1
    R_j = Rotation.from_rotvec([0.01, -0.02, 0.03])
    for d in (0.2, 1.0, 2.0):
        pb = _problem_single_edge(350.0, 200.0, d, IDENT, _pose([0, 0, 0], R_j.as_rotvec()))
        t = ba64.edge_terms(pb)
        Kmat = np.array([[320.0, 0, 320.0], [0, 320.0, 240.0], [0, 0, 1]])
        h = Kmat @ R_j.as_matrix().T @ np.linalg.inv(Kmat) @ np.array([350.0, 200.0, 1.0])
        np.testing.assert_allclose(t.proj[0], h[:2] / h[2], atol=1e-10)


def test_validity_rule():
    # point straight ahead at depth 1/d = 2; camera j moved forward by 1.95 -> q_z = 0.05 d < z_min d
    pb = _problem_single_edge(320.0, 240.0, 0.5, IDENT, _pose([0, 0, 1.95]))
    assert not ba64.edge_terms(pb).valid[0]
    pb = _problem_single_edge(320.0, 240.0, 0.5, IDENT, _pose([0, 0, 1.85]))
    assert ba64.edge_terms(pb).valid[0]
    pb = _problem_single_edge(320.0, 240.0, -0.5, IDENT, IDENT)
    assert not ba64.edge_terms(pb).valid[0]


def test_ground_truth_rendering_is_a_fixed_point():
    # the scene generator renders world points by a different route (explicit
    # 3-D points, world-to-camera); eq. 2 in inverse-depth form must agree
    s = tiny_scene(6, 8, seed=3, noise_px=0.0, init="gt")
    pb = ba64.Problem.from_scene(s)
    pb.poses = s.poses_gt.copy(); pb.inv_depth = s.inv_depth_gt.copy(); pb.target = s.target64.copy()
    assert np.abs(ba64.edge_terms(pb).r).max() < 1e-9


# ---------------------------------------------------------------- Jacobians

def _residual(pb, poses, d):
    return ba64.edge_terms(pb, poses, d).r


def _perturb_pose(poses, idx, xi):
    R, t = lie64.pose_to_rt(poses[idx])
    Rn, tn = lie64.retract_right(R, t, xi)
    out = poses.copy()
    out[idx] = lie64.rt_to_pose(Rn[None], tn[None])[0]
    return out


def test_jacobians_match_central_differences():
    s = tiny_scene(4, 5, seed=7)
    pb = ba64.Problem.from_scene(s)
    t = ba64.edge_terms(pb)
    h = 1e-6
    for e in range(0, pb.ii.shape[0], 7):
        i, j, k = pb.ii[e], pb.jj[e], pb.kk[e]
        for a in range(6):
            xi = np.zeros(6); xi[a] = h
            for idx, J in ((i, t.Ji), (j, t.Jj)):
                rp = _residual(pb, _perturb_pose(pb.poses, idx, xi), pb.inv_depth)[e]
                rm = _residual(pb, _perturb_pose(pb.poses, idx, -xi), pb.inv_depth)[e]
                fd = (rp - rm) / (2 * h)
                np.testing.assert_allclose(J[e, :, a], fd, rtol=1e-6, atol=1e-6 * (1 + np.abs(fd).max()))
        dp = pb.inv_depth.copy(); dp[k] += h
        dm = pb.inv_depth.copy(); dm[k] -= h
        fd = (_residual(pb, pb.poses, dp)[e] - _residual(pb, pb.poses, dm)[e]) / (2 * h)
        np.testing.assert_allclose(t.Jd[e], fd, rtol=1e-6, atol=1e-6 * (1 + np.abs(fd).max()))


def test_jacobian_adjoint_identity():
    # J_i = -J_j Ad(T_ji) with Ad = [[R, [t]x R], [0, R]] for xi = (rho, phi)
    s = tiny_scene(4, 5, seed=8)
    pb = ba64.Problem.from_scene(s)
    t = ba64.edge_terms(pb)
    Rji, tji = ba64.relative_poses(pb.poses, pb.ii, pb.jj)
    for e in range(pb.ii.shape[0]):
        R, tt = Rji[e], tji[e]
        Ad = np.zeros((6, 6))
        Ad[:3, :3] = R; Ad[3:, 3:] = R; Ad[:3, 3:] = lie64.hat(tt) @ R
        np.testing.assert_allclose(t.Ji[e], -(t.Jj[e] @ Ad) * 1.0, rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------- normal equations and solve

def _fd_jacobian(pb, poses, d):
    """Dense Jacobian of the stacked residual over (free xi, all depths) by
    central differences of the residual function."""
    nf = pb.n_fixed
    h = 1e-6
    cols = []
    for idx in range(nf, pb.n_frames):
        for a in range(6):
            xi = np.zeros(6); xi[a] = h
            rp = _residual(pb, _perturb_pose(poses, idx, xi), d)
            rm = _residual(pb, _perturb_pose(poses, idx, -xi), d)
            cols.append(((rp - rm) / (2 * h)).reshape(-1))
    for k in range(pb.n_patches):
        dp = d.copy(); dp[k] += h
        dm = d.copy(); dm[k] -= h
        cols.append(((_residual(pb, poses, dp) - _residual(pb, poses, dm)) / (2 * h)).reshape(-1))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("lam", [1e-4, 1e-1])
def test_schur_step_equals_dense_damped_step_from_fd_jacobian(lam):
    s = tiny_scene(4, 5, seed=11)
    pb = ba64.Problem.from_scene(s)
    J = _fd_jacobian(pb, pb.poses, pb.inv_depth)
    W = np.diag(pb.weight.reshape(-1))
    r = ba64.edge_terms(pb).r.reshape(-1)
    H = J.T @ W @ J
    g = J.T @ W @ r
    Ht = H + lam * (np.diag(np.diag(H)) + np.eye(H.shape[0]))
    delta = np.linalg.solve(Ht, -g)
    terms = ba64.edge_terms(pb)
    ne = ba64.normal_equations(pb, terms)
    rs = ba64.reduce(ne, lam)
    dxi = ba64.solve_reduced(rs)
    dd = ba64.back_substitute(ne, rs, dxi)
    np.testing.assert_allclose(np.concatenate([dxi, dd]), delta, rtol=1e-5, atol=1e-7 * np.abs(delta).max())
    np.testing.assert_allclose(ne.H.toarray(), H, rtol=1e-6, atol=1e-6 * np.abs(H).max())


def test_schur_step_equals_dense_solve_exactly():
    s = tiny_scene(5, 6, seed=12)
    pb = ba64.Problem.from_scene(s)
    terms = ba64.edge_terms(pb)
    ne = ba64.normal_equations(pb, terms)
    lam = 1e-4
    H = ne.H.toarray()
    Ht = H + lam * (np.diag(np.diag(H)) + np.eye(H.shape[0]))
    delta = np.linalg.solve(Ht, -ne.g)
    rs = ba64.reduce(ne, lam)
    dxi = ba64.solve_reduced(rs)
    dd = ba64.back_substitute(ne, rs, dxi)
    np.testing.assert_allclose(np.concatenate([dxi, dd]), delta, rtol=1e-9, atol=1e-12 * np.abs(delta).max())


def test_large_damping_limit_is_scaled_gradient_step():
    # lam -> inf: delta -> -g / (lam (diag(H) + 1)); pins the form of the damping
    s = tiny_scene(4, 5, seed=13)
    pb = ba64.Problem.from_scene(s)
    J = _fd_jacobian(pb, pb.poses, pb.inv_depth)
    W = np.diag(pb.weight.reshape(-1))
    r = ba64.edge_terms(pb).r.reshape(-1)
    H = J.T @ W @ J
    g = J.T @ W @ r
    lam = 1e9
    ne = ba64.normal_equations(pb, ba64.edge_terms(pb))
    rs = ba64.reduce(ne, lam)
    dxi = ba64.solve_reduced(rs)
    dd = ba64.back_substitute(ne, rs, dxi)
    limit = -g / (lam * (np.diag(H) + 1.0))
    np.testing.assert_allclose(np.concatenate([dxi, dd]), limit, rtol=1e-4, atol=1e-4 * np.abs(limit).max())


def test_structure_only_step_closed_form():
    # every pose held: each depth takes its own damped 1-D Gauss-Newton step
    s = tiny_scene(4, 5, seed=14)
    pb = ba64.Problem.from_scene(s)
    pb.n_fixed = pb.n_frames
    lam = 1e-3
    h = 1e-6
    d = pb.inv_depth
    r0 = _residual(pb, pb.poses, d)
    P, D, _ = ba64.solve(pb, n_iters=1, lam=lam)
    np.testing.assert_allclose(P, pb.poses, atol=0)
    for k in range(pb.n_patches):
        dp = d.copy(); dp[k] += h
        dm = d.copy(); dm[k] -= h
        jd = (_residual(pb, pb.poses, dp) - _residual(pb, pb.poses, dm)) / (2 * h)
        sel = pb.kk == k
        c = np.sum(pb.weight[sel] * jd[sel] ** 2)
        b = np.sum(pb.weight[sel] * jd[sel] * r0[sel])
        np.testing.assert_allclose(D[k] - d[k], -b / (c * (1 + lam) + lam), rtol=1e-6, atol=1e-10)


# ---------------------------------------------------------------- Gauss-Newton invariants

def test_ground_truth_is_fixed_point():
    s = tiny_scene(6, 8, seed=21, noise_px=0.0, init="gt")
    pb = ba64.Problem.from_scene(s)
    pb.poses = s.poses_gt.copy(); pb.inv_depth = s.inv_depth_gt.copy(); pb.target = s.target64.copy()
    P, D, rep = ba64.solve(pb, n_iters=1)
    assert rep.step_norm[0] < 1e-10 and rep.depth_step_norm[0] < 1e-10


def test_recovers_ground_truth_noise_free():
    s = tiny_scene(6, 8, seed=22, noise_px=0.0)
    pb = ba64.Problem.from_scene(s)
    pb.poses = s.poses.astype(np.float64); pb.poses[: s.n_fixed] = s.poses_gt[: s.n_fixed]
    pb.target = s.target64.copy()
    P, D, rep = ba64.solve(pb, n_iters=30, lam=1e-4)
    dt, dr = ba64.pose_errors(P, s.poses_gt)
    assert dt.max() < 1e-9 and dr.max() < 1e-9
    np.testing.assert_allclose(D, s.inv_depth_gt, rtol=1e-9)


def test_rigid_gauge_equivariance():
    s = tiny_scene(5, 6, seed=23)
    pb = ba64.Problem.from_scene(s)
    P, D, _ = ba64.solve(pb, n_iters=3)
    T_R = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    T_t = np.array([1.0, -2.0, 0.5])
    R0, t0 = lie64.pose_to_rt(pb.poses)
    pb2 = ba64.Problem.from_scene(s)
    pb2.poses = lie64.rt_to_pose(T_R @ R0, t0 @ T_R.T + T_t)
    P2, D2, _ = ba64.solve(pb2, n_iters=3)
    R, t = lie64.pose_to_rt(P)
    R2, t2 = lie64.pose_to_rt(P2)
    np.testing.assert_allclose(R2, T_R @ R, atol=1e-11)
    np.testing.assert_allclose(t2, t @ T_R.T + T_t, atol=1e-11)
    np.testing.assert_allclose(D2, D, rtol=1e-10)


def test_monocular_scale_invariance_without_damping():
    # t -> s t, d -> d / s leaves every residual unchanged (the Sim(3) action on
    # poses and inverse depths); with lam = 0 the iterates transform exactly
    s = tiny_scene(5, 6, seed=24)
    pb = ba64.Problem.from_scene(s)
    P, D, _ = ba64.solve(pb, n_iters=2, lam=0.0)
    sc = 2.5
    pb2 = ba64.Problem.from_scene(s)
    pb2.poses = pb.poses.copy(); pb2.poses[:, :3] *= sc
    pb2.inv_depth = pb.inv_depth / sc
    P2, D2, _ = ba64.solve(pb2, n_iters=2, lam=0.0)
    np.testing.assert_allclose(P2[:, :3], sc * P[:, :3], rtol=1e-9, atol=1e-11)
    dt, dr = ba64.pose_errors(P2, P)
    assert dr.max() < 1e-10
    np.testing.assert_allclose(D2, D / sc, rtol=1e-9)


def test_edge_order_invariance():
    s = tiny_scene(5, 6, seed=25)
    pb = ba64.Problem.from_scene(s)
    P, D, _ = ba64.solve(pb, n_iters=2)
    perm = np.random.default_rng(0).permutation(pb.ii.shape[0])
    pb2 = ba64.Problem.from_scene(s)
    for f in ("ii", "jj", "kk", "target", "weight"):
        setattr(pb2, f, getattr(pb, f)[perm])
    P2, D2, _ = ba64.solve(pb2, n_iters=2)
    np.testing.assert_allclose(P2, P, atol=1e-12)
    np.testing.assert_allclose(D2, D, rtol=1e-11)


def test_duplicated_edge_equals_doubled_weight():
    s = tiny_scene(5, 6, seed=26)
    pb = ba64.Problem.from_scene(s)
    e = 3
    pb2 = ba64.Problem.from_scene(s)
    for f in ("ii", "jj", "kk", "target", "weight"):
        a = getattr(pb, f)
        setattr(pb2, f, np.concatenate([a, a[e:e + 1]]))
    pb3 = ba64.Problem.from_scene(s)
    pb3.weight = pb.weight.copy(); pb3.weight[e] *= 2
    P2, D2, _ = ba64.solve(pb2, n_iters=2)
    P3, D3, _ = ba64.solve(pb3, n_iters=2)
    np.testing.assert_allclose(P2, P3, atol=1e-12)
    np.testing.assert_allclose(D2, D3, rtol=1e-11)


def test_cost_decreases_on_small_configs():
    s = make_config(0)
    P, D, rep = ba64.solve_scene(s)
    assert rep.cost[-1] < rep.cost[0] * 0.01
    assert rep.n_invalid == [0, 0]


# ---------------------------------------------------------------- cost of eq. 3 (hand-worked values)

def _two_camera_problem(targets, weights, depths, pose_j):
    """Two patches of frame 0 seen from frame 1 (one edge each)."""
    P = len(depths)
    centres = np.array([[400.0, 200.0]] * P)
    return ba64.Problem(
        poses=np.stack([IDENT, pose_j]).astype(np.float64), centres=centres,
        inv_depth=np.asarray(depths, dtype=np.float64), ii=np.zeros(P, dtype=np.int64),
        jj=np.ones(P, dtype=np.int64), kk=np.arange(P), target=np.asarray(targets, dtype=np.float64),
        weight=np.asarray(weights, dtype=np.float64), intrinsics=np.array([320.0, 320.0, 320.0, 240.0]),
        n_fixed=0)


def test_cost_single_edge_hand_value():
    # sideways translation b = 0.1, d = 0.5: the centre lands at (384, 200)
    # (u' = u - fx b d).  Target (380, 197): r = (4, 3); w = (0.5, 1):
    # cost = 1/2 (0.5 * 16 + 1 * 9) = 8.5
    pb = _two_camera_problem([[380.0, 197.0]], [[0.5, 1.0]], [0.5], _pose([0.1, 0, 0]))
    t = ba64.edge_terms(pb)
    np.testing.assert_allclose(t.r[0], [4.0, 3.0], atol=1e-12)
    assert abs(ba64.cost(pb, t) - 8.5) < 1e-12
    # only x off the target: r = (4, 0), w = (0.5, 1): cost = 1/2 * 0.5 * 16 = 4
    pb = _two_camera_problem([[380.0, 200.0]], [[0.5, 1.0]], [0.5], _pose([0.1, 0, 0]))
    assert abs(ba64.cost(pb, ba64.edge_terms(pb)) - 4.0) < 1e-12


def test_cost_skips_invalid_edges():
    # edge 0 as above (cost 8.5); edge 1 has a negative inverse depth, so it is
    # invalid and contributes nothing however far its reprojection lands
    pb = _two_camera_problem([[380.0, 197.0], [-5000.0, 9000.0]], [[0.5, 1.0], [1.0, 1.0]], [0.5, -0.5],
                             _pose([0.1, 0, 0]))
    t = ba64.edge_terms(pb)
    assert t.valid.tolist() == [True, False]
    assert abs(ba64.cost(pb, t) - 8.5) < 1e-12


def test_cost_is_zero_at_ground_truth_noise_free():
    s = tiny_scene(6, 8, seed=31, noise_px=0.0, init="gt")
    pb = ba64.Problem.from_scene(s)
    pb.poses = s.poses_gt.copy(); pb.inv_depth = s.inv_depth_gt.copy(); pb.target = s.target64.copy()
    assert ba64.cost(pb, ba64.edge_terms(pb)) < 1e-18 * s.n_edges + 1e-20
    # and equals the hand sum over edges once every target moves by (1, -2) px
    pb.target = s.target64 + np.array([1.0, -2.0])
    want = 0.5 * float(np.sum(pb.weight[:, 0] * 1.0 + pb.weight[:, 1] * 4.0))
    assert abs(ba64.cost(pb, ba64.edge_terms(pb)) - want) < 1e-9 * want


# ---------------------------------------------------------------- full-patch reprojection (eq. 2 per pixel)

def test_reproject_every_pixel_sideways_translation():
    # every pixel of the patch moves by -fx b d along x (one inverse depth per patch)
    b, d = 0.1, 0.5
    pb = _problem_single_edge(400.0, 200.0, d, IDENT, _pose([b, 0, 0]))
    full, valid = ba64.reproject(pb)
    want = pb.patches[0].copy()
    want[..., 0] -= 320.0 * b * d
    np.testing.assert_allclose(full[0], want, atol=1e-12)
    assert valid.all()


def test_reproject_every_pixel_forward_translation():
    # camera moved forward by b along its axis: every pixel scales about the
    # principal point by 1 / (1 - b d)
    b, d = 0.1, 0.5
    pb = _problem_single_edge(400.0, 300.0, d, IDENT, _pose([0, 0, b]))
    full, _ = ba64.reproject(pb)
    want = np.empty_like(pb.patches[0])
    want[..., 0] = 320.0 + (pb.patches[0][..., 0] - 320.0) / (1 - b * d)
    want[..., 1] = 240.0 + (pb.patches[0][..., 1] - 240.0) / (1 - b * d)
    np.testing.assert_allclose(full[0], want, atol=1e-12)


def test_reproject_centre_matches_edge_terms():
    s = tiny_scene(5, 6, seed=32)
    pb = ba64.Problem.from_scene(s)
    full, valid = ba64.reproject(pb)
    t = ba64.edge_terms(pb)
    c = (s.patches.shape[1] - 1) // 2
    np.testing.assert_allclose(full[:, c, c, :], t.proj, atol=1e-9)
    assert (valid == t.valid).all()


def test_levenberg_damping_pins():
    # H + lam I: equals the dense solve of that system, and tends to -g / lam
    s = tiny_scene(4, 5, seed=15)
    pb = ba64.Problem.from_scene(s)
    ne = ba64.normal_equations(pb, ba64.edge_terms(pb))
    H = ne.H.toarray()
    for lam in (1e-3, 1e14):  # the limit needs lam far above H's entries (up to ~1e7 here)
        rs = ba64.reduce(ne, lam, levenberg=True)
        dxi = ba64.solve_reduced(rs)
        dd = ba64.back_substitute(ne, rs, dxi)
        delta = np.concatenate([dxi, dd])
        want = np.linalg.solve(H + lam * np.eye(H.shape[0]), -ne.g)
        np.testing.assert_allclose(delta, want, rtol=1e-8, atol=1e-12 * np.abs(want).max())
        if lam > 1e6:
            np.testing.assert_allclose(delta, -ne.g / lam, rtol=1e-4, atol=1e-4 * np.abs(ne.g / lam).max())


def test_solution_independent_of_frame_numbering():
    # renumbering the free frames permutes the reduced system symmetrically;
    # Gauss-Newton steps (and so the solution) must not depend on it
    from scenes import relabel_frames
    s = tiny_scene(10, 6, seed=12)
    r = relabel_frames(s, seed=3)
    new = r.meta["relabel"]
    P1, D1, _ = ba64.solve_scene(s)
    P2, D2, _ = ba64.solve_scene(r)
    dt, dr = ba64.pose_errors(P1, P2[new])
    assert dt.max() < 1e-10 and dr.max() < 1e-10
    np.testing.assert_allclose(D1, D2, rtol=1e-10)
    assert not np.array_equal(new[s.n_fixed:], np.arange(s.n_fixed, s.n_frames))
