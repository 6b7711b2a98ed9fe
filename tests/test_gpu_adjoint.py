"""GPU parity of the adjoint (dpvba_solve_backward and the autograd layer)
against the float64 gradient oracle (oracle/grad64.py, itself pinned by
central differences).

Tolerances, relative to the largest oracle gradient entry: float64 mode
1e-8 (each iteration's adjoint solves a system with condition number up to
~1e5 at these sizes, so a few 1e-11 per solve, summed over the iterations
and edges).  Float32 mode: a bound derived per scene from the conditioning
of its damped reduced system S: T unrolled iterations take 2T + 1 solves
with S-like systems (forward step, adjoint solve, and the float32 iterate the
Jacobians are evaluated at), each with relative error up to about
kappa(S) eps32; a factor 10 covers the per-edge sums, so
tol32 = 10 (2T + 1) kappa(S) eps32 (about 5e-4 for a 22-frame window,
kappa(S) = 161).

The supervision loss of the cfg3 windows is the pose loss
sum ||t - t_gt||^2 + ||Log(R_gt^T R)||^2 over free poses; other tests use a
loss that also touches the inverse depths.
"""
import numpy as np
import pytest
import torch

from oracle import grad64
from scenes import make_config, make_window, relabel_frames, tiny_scene

pytestmark = pytest.mark.gpu

TOL64 = 1e-8
EPS32 = float(np.finfo(np.float32).eps)


def _tol32(s):
    from oracle import ba64
    pb = ba64.Problem.from_scene(s)
    rs = ba64.reduce(ba64.normal_equations(pb, ba64.edge_terms(pb, z_min=s.z_min)), s.lam)
    return 10 * (2 * s.n_iters + 1) * float(np.linalg.cond(rs.S)) * EPS32


@pytest.fixture(scope="module")
def dp():
    import paper_2408_01654_amd as dp
    return dp


@pytest.fixture(scope="module")
def ctx(dp):
    c = dp.Context(0)
    yield c
    c.close()


def _log(msg):
    print(msg, flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _gpu_backward64(dp, ctx, s, gp, gd, n_iters):
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g)
    p0 = torch.as_tensor(s.poses, dtype=torch.float64).cuda().contiguous()
    d0 = torch.as_tensor(s.inv_depth, dtype=torch.float64).cuda().contiguous()
    gpt = None if gp is None else torch.as_tensor(gp).cuda().contiguous()
    gdt = None if gd is None else torch.as_tensor(gd).cuda().contiguous()
    gt, gw = ctx.solve_backward(g, p0, d0, gpt, gdt, n_iters=n_iters, lam=s.lam, z_min=s.z_min, precision=dp.FP64)
    torch.cuda.synchronize()
    return gt.cpu().numpy(), gw.cpu().numpy()


def _drop_edges_of_patch(s, k):
    keep = s.kk != k
    s.ii, s.jj, s.kk = s.ii[keep], s.jj[keep], s.kk[keep]
    s.target, s.weight = s.target[keep], s.weight[keep]
    return s


def _duplicate_edges(s, idx):
    for name in ("ii", "jj", "kk", "target", "weight"):
        a = getattr(s, name)
        setattr(s, name, np.concatenate([a, a[idx]], 0))
    return s


def _behind_camera(s, k):
    s.inv_depth = s.inv_depth.copy()
    s.inv_depth[k] = -0.2
    return s


SCENES = [
    ("tiny", lambda: tiny_scene(5, 5, seed=41), None),
    ("held3", lambda: tiny_scene(6, 4, seed=43, n_fixed=2), 3),
    ("edgeless", lambda: _drop_edges_of_patch(tiny_scene(5, 5, seed=45), 7), None),
    ("duplicates", lambda: _duplicate_edges(tiny_scene(5, 5, seed=46), np.arange(0, 40, 3)), None),
    ("invalid", lambda: _behind_camera(tiny_scene(5, 5, seed=47), 3), None),
    ("cfg0", lambda: make_config(0), None),
    ("window", lambda: make_window(0), None),
    # 60 frames, 58 free: n = 348, the blocked factorisation of the large path
    ("blocked", lambda: tiny_scene(60, 12, seed=4, radius=5, trajectory="forward"), None),
    # the same with its free frames numbered at random: the analysis factors
    # the reduced system in a fill-reducing order, the adjoint solves included
    ("relabelled", lambda: relabel_frames(tiny_scene(60, 12, seed=4, radius=5, trajectory="forward"), seed=5),
     None),
]


@pytest.mark.parametrize("name,mk,n_iters", SCENES, ids=[x[0] for x in SCENES])
def test_backward_matches_gradient_oracle_fp64(dp, ctx, name, mk, n_iters):
    s = mk()
    nit = s.n_iters if n_iters is None else n_iters
    _log(f"adjoint fp64 {name} N={s.n_frames} E={s.n_edges} iters={nit}")
    L, gt_o, gw_o, gp_o, gd_o = grad64.loss_and_grads(s, n_iters=nit)
    gt, gw = _gpu_backward64(dp, ctx, s, gp_o, gd_o, nit)
    et, ew = _rel(gt, gt_o), _rel(gw, gw_o)
    _log(f"  target rel {et:.3e}  weight rel {ew:.3e}  max|g| {np.abs(gt_o).max():.3e} {np.abs(gw_o).max():.3e}")
    assert et < TOL64 and ew < TOL64
    if name == "invalid":
        dead = s.kk == 3
        assert np.all(gt[dead] == 0) and np.all(gw[dead] == 0)


def test_backward_depth_only_and_zero_iterations(dp, ctx):
    s = tiny_scene(5, 5, seed=48)
    ref = torch.as_tensor(s.inv_depth_gt, dtype=torch.float64)
    loss = lambda poses, d: ((d - ref) ** 2).sum()
    L, gt_o, gw_o, gp_o, gd_o = grad64.loss_and_grads(s, loss_fn=loss)
    assert np.all(gp_o == 0)
    gt, gw = _gpu_backward64(dp, ctx, s, None, gd_o, s.n_iters)
    _log(f"adjoint depth-only: target rel {_rel(gt, gt_o):.3e} weight rel {_rel(gw, gw_o):.3e}")
    assert _rel(gt, gt_o) < TOL64 and _rel(gw, gw_o) < TOL64
    gt0, gw0 = _gpu_backward64(dp, ctx, s, gp_o, gd_o, 0)
    assert np.all(gt0 == 0) and np.all(gw0 == 0)


def test_backward_is_deterministic(dp, ctx):
    s = make_config(0)
    L, gt_o, gw_o, gp_o, gd_o = grad64.loss_and_grads(s)
    a = _gpu_backward64(dp, ctx, s, gp_o, gd_o, s.n_iters)
    b = _gpu_backward64(dp, ctx, s, gp_o, gd_o, s.n_iters)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("mk", [lambda: tiny_scene(5, 5, seed=41), lambda: make_window(0)], ids=["tiny", "window"])
def test_autograd_layer_fp32(dp, ctx, mk):
    s = mk()
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g)
    target = g.target.clone().requires_grad_(True)
    weight = g.weight.clone().requires_grad_(True)
    p0 = torch.as_tensor(s.poses, dtype=torch.float32).cuda()
    d0 = torch.as_tensor(s.inv_depth, dtype=torch.float32).cuda()
    poses, d = dp.bundle_adjust(ctx, g, p0, d0, target, weight, n_iters=s.n_iters, lam=s.lam, z_min=s.z_min)
    ref_p = torch.as_tensor(s.poses_gt, dtype=torch.float32).cuda()
    ref_d = torch.as_tensor(s.inv_depth_gt, dtype=torch.float32).cuda()
    loss = grad64.pose_depth_loss(poses, d, ref_p, ref_d, s.n_fixed)
    loss.backward()
    L, gt_o, gw_o, _, _ = grad64.loss_and_grads(s)
    et = _rel(target.grad.double().cpu().numpy(), gt_o)
    ew = _rel(weight.grad.double().cpu().numpy(), gw_o)
    _log(f"autograd fp32 {s.name}: loss {float(loss):.6e} vs {L:.6e}; target rel {et:.3e} weight rel {ew:.3e}")
    tol = _tol32(s)
    _log(f"  float32 tolerance {tol:.3e}")
    assert abs(float(loss) - L) <= 1e-3 * max(1.0, abs(L))
    assert et < tol and ew < tol


@pytest.mark.parametrize("i", range(16))
def test_adjoint_windows_pose_loss_fp64(dp, ctx, i):
    """Every window of the 16-window adjoint workload (12-22 frames x 64-96
    patches), supervised with the pose loss, against the gradient oracle."""
    s = make_config(3, i)
    loss = grad64.scene_pose_loss(s)
    L, gt_o, gw_o, gp_o, gd_o = grad64.loss_and_grads(s, loss_fn=loss)
    assert np.all(gd_o == 0)
    gt, gw = _gpu_backward64(dp, ctx, s, gp_o, None, s.n_iters)
    et, ew = _rel(gt, gt_o), _rel(gw, gw_o)
    _log(f"window {i} F={s.n_frames} E={s.n_edges}: target rel {et:.3e} weight rel {ew:.3e}")
    assert et < TOL64 and ew < TOL64


def test_adjoint_levenberg_fp64(dp, ctx):
    s = tiny_scene(5, 5, seed=51)
    s.lam = 1e-2
    L, gt_o, gw_o, gp_o, gd_o = grad64.loss_and_grads(s, levenberg=True)
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g)
    p0 = torch.as_tensor(s.poses, dtype=torch.float64).cuda().contiguous()
    d0 = torch.as_tensor(s.inv_depth, dtype=torch.float64).cuda().contiguous()
    gt, gw = ctx.solve_backward(g, p0, d0, torch.as_tensor(gp_o).cuda(), torch.as_tensor(gd_o).cuda(),
                                n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, precision=dp.FP64,
                                flags=dp.binding.FLAG_LEVENBERG)
    et, ew = _rel(gt.cpu().numpy(), gt_o), _rel(gw.cpu().numpy(), gw_o)
    _log(f"adjoint levenberg: target rel {et:.3e} weight rel {ew:.3e}")
    assert et < TOL64 and ew < TOL64


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_many_problems_concurrently_match_one_by_one(dp, prec):
    # dpvba_solve_many / dpvba_solve_backward_many run four windows on their
    # contexts' own streams at once; each problem's results must be those of
    # its own call, bit for bit (same kernels, fixed summation orders)
    P = dp.FP64 if prec == "fp64" else dp.FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    scenes = [make_config(3, i) for i in range(4)]
    ctxs = [dp.Context(0) for _ in scenes]
    try:
        gs = [dp.GraphTensors.from_scene(s) for s in scenes]
        for c, g in zip(ctxs, gs):
            c.analyze(g)
        p0 = [torch.as_tensor(s.poses, dtype=dt).cuda().contiguous() for s in scenes]
        d0 = [torch.as_tensor(s.inv_depth, dtype=dt).cuda().contiguous() for s in scenes]
        kw = dict(n_iters=2, lam=scenes[0].lam, z_min=scenes[0].z_min, precision=P)
        pm, dm = [p.clone() for p in p0], [d.clone() for d in d0]
        dp.solve_many(ctxs, gs, pm, dm, **kw)
        gen = torch.Generator().manual_seed(7)
        gp = [torch.randn(p.shape, generator=gen, dtype=dt).cuda() for p in p0]
        gd = [None if i == 2 else torch.randn(d.shape, generator=gen, dtype=dt).cuda() for i, d in enumerate(d0)]
        gt, gw = dp.solve_backward_many(ctxs, gs, p0, d0, gp, gd, **kw)
        torch.cuda.synchronize()
        for i, (c, g) in enumerate(zip(ctxs, gs)):
            p1, d1 = p0[i].clone(), d0[i].clone()
            c.solve(g, p1, d1, report=False, **kw)
            t1, w1 = c.solve_backward(g, p0[i], d0[i], gp[i], gd[i], **kw)
            torch.cuda.synchronize()
            _log(f"many {prec} window {i}: E={g.ii.shape[0]}")
            assert torch.equal(pm[i], p1) and torch.equal(dm[i], d1)
            assert torch.equal(gt[i], t1) and torch.equal(gw[i], w1)
    finally:
        for c in ctxs:
            c.close()


def test_autograd_layer_many_fp32(dp):
    # the layer over several windows (forwards and adjoints concurrent)
    # against the float64 gradient oracle of each window
    scenes = [make_config(3, i) for i in range(3)]
    ctxs = [dp.Context(0) for _ in scenes]
    try:
        gs = [dp.GraphTensors.from_scene(s) for s in scenes]
        for c, g in zip(ctxs, gs):
            c.analyze(g)
        tg = [g.target.clone().requires_grad_(True) for g in gs]
        wg = [g.weight.clone().requires_grad_(True) for g in gs]
        p0 = [torch.as_tensor(s.poses, dtype=torch.float32).cuda() for s in scenes]
        d0 = [torch.as_tensor(s.inv_depth, dtype=torch.float32).cuda() for s in scenes]
        s0 = scenes[0]
        poses, ds = dp.bundle_adjust_many(ctxs, gs, p0, d0, tg, wg, n_iters=s0.n_iters, lam=s0.lam, z_min=s0.z_min)
        loss = sum(grad64.pose_depth_loss(p, d, torch.as_tensor(s.poses_gt, dtype=torch.float32).cuda(),
                                          torch.as_tensor(s.inv_depth_gt, dtype=torch.float32).cuda(), s.n_fixed)
                   for p, d, s in zip(poses, ds, scenes))
        loss.backward()
        for i, s in enumerate(scenes):
            L, gt_o, gw_o, _, _ = grad64.loss_and_grads(s)
            et = _rel(tg[i].grad.double().cpu().numpy(), gt_o)
            ew = _rel(wg[i].grad.double().cpu().numpy(), gw_o)
            tol = _tol32(s)
            _log(f"layer many, window {i}: target rel {et:.3e} weight rel {ew:.3e} (tol {tol:.3e})")
            assert et < tol and ew < tol
    finally:
        for c in ctxs:
            c.close()
