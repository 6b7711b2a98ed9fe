"""Float64 Gauss-Newton bundle adjustment over a patch graph: the oracle.

Test infrastructure only (see the package docstring).

Follows the paper's problem statement: the patch of eq. (1) with one inverse
depth per patch, the reprojection of eq. (2), and the confidence-weighted
least-squares objective of eq. (3); the Schur elimination of the depths and
the Cholesky solve of the pose block follow Appendix A.  The readings taken
where the paper is silent are:

* only the patch centre enters the residual; the full p x p reprojection is
  available separately (``reproject``);
* cost = 1/2 sum_e sum_c w_ec r_ec^2 (confidences multiply the squares);
* poses are camera-to-world, perturbed on the right, G <- G Exp(xi),
  xi = (rho, phi), with the full SE(3) exponential;
* an edge is valid iff d_k > 0 and q_z > z_min d_k; invalid edges contribute
  nothing and are counted;
* damping H~ = H + lam (Diag(H) + I) on the full system, fixed lam, no
  step rejection, a fixed number of iterations;
* poses [0, n_fixed) are held; every depth is free.

The computation is written as its definition: per-edge residuals and
Jacobians, the sparse Jacobian J over the free variables, H = J^T W J and
g = J^T W r, then the Schur complement and a Cholesky factorisation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import lie64


@dataclass
class Problem:
    """One BA problem in float64 (inputs promoted exactly from float32)."""

    poses: np.ndarray      # [N,7]
    centres: np.ndarray    # [P,2] patch centre pixels
    inv_depth: np.ndarray  # [P]
    ii: np.ndarray
    jj: np.ndarray
    kk: np.ndarray
    target: np.ndarray     # [E,2]
    weight: np.ndarray     # [E,2]
    intrinsics: np.ndarray  # fx, fy, cx, cy
    n_fixed: int
    patches: np.ndarray | None = None  # [P,p,p,2] (for the full-patch reprojection)

    @staticmethod
    def from_scene(s) -> "Problem":
        p = s.patches.shape[1]
        c = (p - 1) // 2
        return Problem(
            poses=s.poses.astype(np.float64), centres=s.patches[:, c, c, :].astype(np.float64),
            inv_depth=s.inv_depth.astype(np.float64), ii=s.ii.astype(np.int64),
            jj=s.jj.astype(np.int64), kk=s.kk.astype(np.int64),
            target=s.target.astype(np.float64), weight=s.weight.astype(np.float64),
            intrinsics=s.intrinsics.astype(np.float64), n_fixed=int(s.n_fixed),
            patches=s.patches.astype(np.float64))

    @property
    def n_frames(self):
        return self.poses.shape[0]

    @property
    def n_patches(self):
        return self.inv_depth.shape[0]


@dataclass
class EdgeTerms:
    q: np.ndarray        # [E,3] point in the target camera (homogeneous, scale d)
    proj: np.ndarray     # [E,2] reprojected centre
    r: np.ndarray        # [E,2] residual proj - target
    valid: np.ndarray    # [E] bool
    Ji: np.ndarray       # [E,2,6] d r / d xi_i
    Jj: np.ndarray       # [E,2,6] d r / d xi_j
    Jd: np.ndarray       # [E,2]   d r / d d_k


def relative_poses(poses, ii, jj):
    """T_ji = G_j^-1 G_i for every edge (eq. 2): R = R_j^T R_i, t = R_j^T (t_i - t_j)."""
    R, t = lie64.pose_to_rt(poses)
    Rj_T = np.swapaxes(R[jj], -1, -2)
    return Rj_T @ R[ii], np.einsum("eab,eb->ea", Rj_T, t[ii] - t[jj])


def inverse_projection(pix, intrinsics):
    """Pi^-1 up to scale: the ray (x^, 1) of pixels [..., 2]."""
    fx, fy, cx, cy = intrinsics
    return np.stack([(pix[..., 0] - cx) / fx, (pix[..., 1] - cy) / fy, np.ones(pix.shape[:-1])], axis=-1)


def edge_terms(pb: Problem, poses=None, inv_depth=None, z_min=0.1) -> EdgeTerms:
    """Per-edge reprojection, residual, validity and analytic Jacobians.

    With T_ji = (R, t): q = R x^ + t d (the homogeneous transfer of eq. 2 in
    inverse-depth form), pi = (fx qx/qz + cx, fy qy/qz + cy).  Right
    perturbations give
      J_d = Jpi t,  J_j = Jpi [ -d I | [q]_x ],  J_i = Jpi R [ d I | -[x^]_x ].
    """
    poses = pb.poses if poses is None else poses
    d_all = pb.inv_depth if inv_depth is None else inv_depth
    fx, fy, cx, cy = pb.intrinsics
    Rji, tji = relative_poses(poses, pb.ii, pb.jj)
    xh = inverse_projection(pb.centres[pb.kk], pb.intrinsics)
    d = d_all[pb.kk]
    q = np.einsum("eab,eb->ea", Rji, xh) + tji * d[:, None]
    valid = (d > 0) & (q[:, 2] > z_min * d)
    z = np.where(valid, q[:, 2], 1.0)
    proj = np.stack([fx * q[:, 0] / z + cx, fy * q[:, 1] / z + cy], axis=1)
    r = proj - pb.target
    E = q.shape[0]
    Jpi = np.zeros((E, 2, 3))
    Jpi[:, 0, 0] = fx / z
    Jpi[:, 0, 2] = -fx * q[:, 0] / (z * z)
    Jpi[:, 1, 1] = fy / z
    Jpi[:, 1, 2] = -fy * q[:, 1] / (z * z)
    Jd = np.einsum("eab,eb->ea", Jpi, tji)
    Mj = np.concatenate([-d[:, None, None] * np.eye(3), lie64.hat(q)], axis=2)
    Mi = np.concatenate([d[:, None, None] * np.eye(3), -lie64.hat(xh)], axis=2)
    Jj = Jpi @ Mj
    Ji = Jpi @ Rji @ Mi
    return EdgeTerms(q=q, proj=proj, r=r, valid=valid, Ji=Ji, Jj=Jj, Jd=Jd)


def reproject(pb: Problem, poses=None, inv_depth=None, z_min=0.1):
    """Full p x p reprojection of every edge's patch into its target frame
    (eq. 2 applied to each pixel with the patch's one inverse depth).
    Returns coords [E,p,p,2] and the centre validity [E]."""
    poses = pb.poses if poses is None else poses
    d_all = pb.inv_depth if inv_depth is None else inv_depth
    fx, fy, cx, cy = pb.intrinsics
    Rji, tji = relative_poses(poses, pb.ii, pb.jj)
    xh = inverse_projection(pb.patches[pb.kk], pb.intrinsics)          # [E,p,p,3]
    d = d_all[pb.kk]
    q = np.einsum("eab,exyb->exya", Rji, xh) + tji[:, None, None, :] * d[:, None, None, None]
    out = np.stack([fx * q[..., 0] / q[..., 2] + cx, fy * q[..., 1] / q[..., 2] + cy], axis=-1)
    c = (pb.patches.shape[1] - 1) // 2
    valid = (d > 0) & (q[:, c, c, 2] > z_min * d)
    return out, valid


def cost(pb: Problem, terms: EdgeTerms) -> float:
    """1/2 sum over valid edges of w_x r_x^2 + w_y r_y^2 (eq. 3, weights multiply)."""
    wr2 = np.sum(pb.weight * terms.r * terms.r, axis=1)
    return 0.5 * float(np.sum(np.where(terms.valid, wr2, 0.0)))


@dataclass
class NormalEquations:
    n_pose: int          # 6 * free poses
    B: np.ndarray        # [n,n] pose-pose block of H (undamped)
    E: sp.csr_matrix     # [n,P] pose-depth block
    C: np.ndarray        # [P] depth diagonal
    v: np.ndarray        # [n] pose part of g
    w: np.ndarray        # [P] depth part of g
    H: sp.csr_matrix     # full H
    g: np.ndarray        # full g
    J: sp.csr_matrix     # [2E, n+P]


def jacobian_matrix(pb: Problem, terms: EdgeTerms) -> sp.csr_matrix:
    """Sparse Jacobian of the stacked residuals [r_0x, r_0y, r_1x, ...] with
    respect to (xi of free poses, depths); fixed poses are dropped and invalid
    edges contribute zero rows."""
    E = pb.ii.shape[0]
    nf = pb.n_fixed
    n = 6 * (pb.n_frames - nf)
    rows, cols, vals = [], [], []
    m = terms.valid.astype(np.float64)
    base_rows = 2 * np.arange(E)
    for c in range(2):
        r_idx = base_rows + c
        for pose, Jx in ((pb.ii, terms.Ji), (pb.jj, terms.Jj)):
            free = pose >= nf
            for a in range(6):
                rows.append(r_idx[free])
                cols.append(6 * (pose[free] - nf) + a)
                vals.append(Jx[free, c, a] * m[free])
        rows.append(r_idx)
        cols.append(n + pb.kk)
        vals.append(terms.Jd[:, c] * m)
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * E, n + pb.n_patches))


def normal_equations(pb: Problem, terms: EdgeTerms) -> NormalEquations:
    """H = J^T W J, g = J^T W r with W = diag(w) (eq. 3)."""
    J = jacobian_matrix(pb, terms)
    wflat = pb.weight.reshape(-1)
    rflat = np.where(terms.valid[:, None], terms.r, 0.0).reshape(-1)
    JtW = (J.T @ sp.diags(wflat)).tocsr()
    H = (JtW @ J).tocsr()
    g = JtW @ rflat
    n = 6 * (pb.n_frames - pb.n_fixed)
    B = H[:n, :n].toarray()
    Ecoup = H[:n, n:].tocsr()
    D = H[n:, n:].tocsr()
    C = D.diagonal()
    off = D - sp.diags(C)
    if off.count_nonzero():
        raise AssertionError("depth block of H is not diagonal")
    return NormalEquations(n_pose=n, B=B, E=Ecoup, C=C, v=g[:n], w=g[n:], H=H, g=g, J=J)


@dataclass
class ReducedSystem:
    S: np.ndarray      # [n,n] Schur complement of the damped system
    s: np.ndarray      # [n]
    Ct: np.ndarray     # [P] damped depth diagonal
    Bt_diag: np.ndarray


def reduce(ne: NormalEquations, lam: float, levenberg: bool = False) -> ReducedSystem:
    """Damp H~ = H + lam (Diag(H) + I) (Levenberg-Marquardt; with
    levenberg=True the plain H + lam I), then eliminate the depths:
    S = B~ - E C~^-1 E^T, s = -v + E C~^-1 w."""
    mq = 0.0 if levenberg else 1.0
    Bt = ne.B + lam * np.diag(mq * np.diag(ne.B) + 1.0)
    Ct = ne.C + lam * (mq * ne.C + 1.0)
    Einv = ne.E @ sp.diags(1.0 / Ct)
    S = Bt - (Einv @ ne.E.T).toarray()
    s = -ne.v + Einv @ ne.w
    return ReducedSystem(S=S, s=s, Ct=Ct, Bt_diag=np.diag(Bt).copy())


def solve_reduced(rs: ReducedSystem):
    """Cholesky S = L L^T and the two triangular solves for the pose step."""
    if rs.S.shape[0] == 0:
        return np.zeros(0)
    cf = scipy.linalg.cho_factor(rs.S, lower=True, check_finite=True)
    return scipy.linalg.cho_solve(cf, rs.s)


def back_substitute(ne: NormalEquations, rs: ReducedSystem, dxi: np.ndarray):
    """Depth step dd = C~^-1 (-w - E^T dxi)."""
    return (-ne.w - ne.E.T @ dxi) / rs.Ct


def apply_step(pb: Problem, poses, inv_depth, dxi, dd):
    """Right retraction of the free poses, additive depth update."""
    nf = pb.n_fixed
    R, t = lie64.pose_to_rt(poses)
    xi = dxi.reshape(-1, 6)
    Rn, tn = lie64.retract_right(R[nf:], t[nf:], xi)
    out = poses.copy()
    out[nf:] = lie64.rt_to_pose(Rn, tn)
    return out, inv_depth + dd


@dataclass
class Report:
    cost: list = field(default_factory=list)         # n_iters + 1 entries
    step_norm: list = field(default_factory=list)    # ||dxi|| per iteration
    depth_step_norm: list = field(default_factory=list)
    n_invalid: list = field(default_factory=list)
    min_pivot_ratio: list = field(default_factory=list)


def gn_iteration(pb: Problem, poses, inv_depth, lam=1e-4, z_min=0.1, report=None, levenberg=False):
    terms = edge_terms(pb, poses, inv_depth, z_min)
    ne = normal_equations(pb, terms)
    rs = reduce(ne, lam, levenberg)
    dxi = solve_reduced(rs)
    dd = back_substitute(ne, rs, dxi)
    if report is not None:
        report.cost.append(cost(pb, terms))
        report.step_norm.append(float(np.linalg.norm(dxi)))
        report.depth_step_norm.append(float(np.linalg.norm(dd)))
        report.n_invalid.append(int(np.sum(~terms.valid)))
    return apply_step(pb, poses, inv_depth, dxi, dd)


def solve(pb: Problem, n_iters=2, lam=1e-4, z_min=0.1, levenberg=False):
    """Fixed-count Gauss-Newton; returns (poses [N,7], inv_depth [P], report)."""
    rep = Report()
    poses, d = pb.poses.copy(), pb.inv_depth.copy()
    for _ in range(n_iters):
        poses, d = gn_iteration(pb, poses, d, lam, z_min, rep, levenberg)
    rep.cost.append(cost(pb, edge_terms(pb, poses, d, z_min)))
    return poses, d, rep


def solve_scene(scene, n_iters=None, lam=None, z_min=None, levenberg=False):
    pb = Problem.from_scene(scene)
    return solve(pb, scene.n_iters if n_iters is None else n_iters,
                 scene.lam if lam is None else lam, scene.z_min if z_min is None else z_min, levenberg)


def pose_errors(poses_a, poses_b):
    """Per-pose translation error (m) and rotation error ||Log(R_a^T R_b)|| (rad)."""
    Ra, ta = lie64.pose_to_rt(poses_a)
    Rb, tb = lie64.pose_to_rt(poses_b)
    dt = np.linalg.norm(ta - tb, axis=-1)
    dr = np.linalg.norm(lie64.so3_log(np.swapaxes(Ra, -1, -2) @ Rb), axis=-1)
    return dt, dr
