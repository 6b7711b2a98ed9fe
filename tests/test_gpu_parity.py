"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: float64 mode 1e-9 (pose translation in scene units, rotation
in rad, inverse depth relative); float32 mode 1e-4 on the same quantities.
The reduced camera system itself (assembly + Schur elimination) is compared
element-wise, relative to its largest entry.
"""
import numpy as np
import pytest
import torch

from oracle import ba64
from scenes import make_config, make_window, tiny_scene
from scenes.patchgraph import Scene

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4, "mixed": 1e-4}
PREC = {"fp64": 2, "mixed": 1, "fp32": 0}


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


def _gpu_solve(dp, ctx, s: Scene, precision, n_iters=None, lam=None, keep_order=False):
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g, keep_order=keep_order)
    dt = torch.float64 if precision == dp.FP64 else torch.float32
    poses = torch.as_tensor(s.poses, dtype=dt).cuda().contiguous()
    depth = torch.as_tensor(s.inv_depth, dtype=dt).cuda().contiguous()
    _log(f"  gpu solve {s.name} precision={precision}")
    rep = ctx.solve(g, poses, depth, n_iters=s.n_iters if n_iters is None else n_iters,
                    lam=s.lam if lam is None else lam, z_min=s.z_min, precision=precision)
    return poses.double().cpu().numpy(), depth.double().cpu().numpy(), rep


def _compare(s, P, D, Po, Do, tol, what):
    dt, dr = ba64.pose_errors(P, Po)
    rel = np.abs(D - Do) / np.maximum(np.abs(Do), 1e-12)
    _log(f"{what}: max dt {dt.max():.3e} dr {dr.max():.3e} depth rel {rel.max():.3e}")
    assert dt.max() < tol and dr.max() < tol and rel.max() < tol, what


SMALL_SCENES = [
    lambda: tiny_scene(4, 6, seed=1),
    lambda: tiny_scene(6, 9, seed=2, radius=2),
    lambda: make_config(0),
    lambda: make_window(0),
    lambda: make_window(537),
]


@pytest.mark.parametrize("mk", SMALL_SCENES)
@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_reduced_system_matches_oracle(dp, ctx, mk, prec):
    s = mk()
    _log(f"reduced system {s.name} {prec}")
    pb = ba64.Problem.from_scene(s)
    ne = ba64.normal_equations(pb, ba64.edge_terms(pb, z_min=s.z_min))
    rs = ba64.reduce(ne, s.lam)
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g)
    precision = PREC[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    poses = torch.as_tensor(s.poses, dtype=dt).cuda()
    depth = torch.as_tensor(s.inv_depth, dtype=dt).cuda()
    S, sv, cost = ctx.reduced_system(g, poses, depth, lam=s.lam, z_min=s.z_min, precision=precision)
    assert S.dtype == (torch.float32 if prec == "fp32" else torch.float64)
    S = S.double().cpu().numpy(); sv = sv.double().cpu().numpy()
    # float64: rounding of sums with cancellation (terms up to ~1e3 x |S|);
    # mixed: float32 per-tile shares, so the float32 bound applies
    tol = 1e-11 if prec == "fp64" else 2e-5
    errS = np.abs(S - rs.S).max() / np.abs(rs.S).max()
    errs = np.abs(sv - rs.s).max() / np.abs(rs.s).max()
    oc = ba64.cost(pb, ba64.edge_terms(pb, z_min=s.z_min))
    _log(f"  S rel {errS:.3e}  s rel {errs:.3e}  cost {cost.item():.6e} vs {oc:.6e}")
    assert errS < tol and errs < tol
    assert abs(cost.item() - oc) <= (1e-12 if prec == "fp64" else 1e-5) * oc


@pytest.mark.parametrize("mk", SMALL_SCENES)
@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_solve_matches_oracle(dp, ctx, mk, prec):
    s = mk()
    _log(f"solve {s.name} {prec}")
    Po, Do, rep_o = ba64.solve_scene(s)
    P, D, rep = _gpu_solve(dp, ctx, s, PREC[prec])
    assert rep["status"] == 0
    if prec == "mixed":
        _log(f"  refine resid {rep['refine_resid']} fallback {rep['fp64_fallback']}")
        assert all(r <= 1e-8 or f == 1 for r, f in zip(rep["refine_resid"], rep["fp64_fallback"]))
    else:
        assert rep["refine_resid"] == [0.0] * s.n_iters and rep["fp64_fallback"] == [0] * s.n_iters
    assert rep["n_invalid"] == rep_o.n_invalid
    np.testing.assert_allclose(rep["cost"], rep_o.cost, rtol=1e-9 if prec == "fp64" else 1e-3)
    _compare(s, P, D, Po, Do, TOL[prec], f"{s.name} {prec}")


@pytest.mark.parametrize("frames", [60, 52])
def test_large_reduced_system_uses_blocked_factorisation(dp, ctx, frames):
    # 60 frames, 58 free: n = 348 (six 64-row blocks: three pairs of the
    # triangular-solve chain); 52 frames: n = 300 (five blocks: the last pair
    # has one block); both above the single-workgroup limit
    s = tiny_scene(frames, 12, seed=4, radius=5, trajectory="forward")
    _log(f"blocked path {s.name} E={s.n_edges}")
    Po, Do, _ = ba64.solve_scene(s)
    for prec in ("fp64", "mixed", "fp32"):
        P, D, rep = _gpu_solve(dp, ctx, s, PREC[prec])
        assert rep["status"] == 0
        _compare(s, P, D, Po, Do, TOL[prec], f"blocked {prec}")


def test_envelope_limited_factor_on_a_loop(dp, ctx):
    # 200 keyframes on the global-BA circle (1.58 laps) with 48 patches each:
    # the proximity loops couple each pose with the same place one lap later,
    # so the early panels of the factor reach only part of the n = 1194 rows
    # and the trailing updates stop at their reach; the result must still
    # match the float64 oracle
    # (in the keyframes' own order and in the analysis' fill-reducing order)
    from scenes import make_sweep
    s = make_sweep(200, total_patches=9600)
    _log(f"envelope {s.name} E={s.n_edges}")
    Po, Do, _ = ba64.solve_scene(s)
    for keep in (True, False):
        for prec in ("fp32", "mixed", "fp64"):
            P, D, rep = _gpu_solve(dp, ctx, s, PREC[prec], keep_order=keep)
            assert rep["status"] == 0
            _compare(s, P, D, Po, Do, TOL[prec], f"envelope {prec} keep_order={keep}")


def _envelope_blocks(s, order):
    """Sum over block rows of the squared envelope width (in pose blocks)
    of the reduced system factored in `order` (block row p = free pose
    order[p]); two free poses are coupled when a patch links them."""
    nf = s.n_fixed
    pos = np.argsort(order)
    first = pos.copy()
    for k in np.unique(s.kk):
        fr = np.unique(np.r_[s.ii[s.kk == k], s.jj[s.kk == k]])
        fr = fr[fr >= nf] - nf
        if len(fr):
            first[fr] = np.minimum(first[fr], pos[fr].min())
    return float(np.sum((pos - first + 1.0) ** 2))


def test_fill_reducing_order_on_relabelled_frames(dp, ctx):
    # a banded problem (forward motion, targets within 5 frames) with its
    # free frames numbered at random: in that numbering the envelope spans
    # the whole system; the analysis must find an order with a far smaller
    # one, report it, and every precision must still match the oracle
    from scenes import relabel_frames
    s = relabel_frames(tiny_scene(60, 12, seed=4, radius=5, trajectory="forward"), seed=5)
    nfree = s.n_frames - s.n_fixed
    Po, Do, _ = ba64.solve_scene(s)
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g, keep_order=True)
    assert np.array_equal(ctx.system_order(), np.arange(nfree))
    ctx.analyze(g)
    order = ctx.system_order()
    assert np.array_equal(np.sort(order), np.arange(nfree))
    e_nat, e_sys = _envelope_blocks(s, np.arange(nfree)), _envelope_blocks(s, order)
    _log(f"relabelled: envelope (blocks^2) natural {e_nat:.0f}, system order {e_sys:.0f}")
    assert e_sys < 0.25 * e_nat
    for keep in (False, True):
        for prec in ("fp32", "mixed", "fp64"):
            P, D, rep = _gpu_solve(dp, ctx, s, PREC[prec], keep_order=keep)
            assert rep["status"] == 0
            _compare(s, P, D, Po, Do, TOL[prec], f"relabelled {prec} keep_order={keep}")


def test_reproject_matches_oracle(dp, ctx):
    s = make_config(0)
    pb = ba64.Problem.from_scene(s)
    coords_o, valid_o = ba64.reproject(pb, z_min=0.1)
    g = dp.GraphTensors.from_scene(s)
    poses = torch.as_tensor(s.poses).cuda()
    depth = torch.as_tensor(s.inv_depth).cuda()
    coords, valid = ctx.reproject(g, poses, depth, z_min=0.1)
    err = np.abs(coords.double().cpu().numpy() - coords_o).max()
    _log(f"reproject max err {err:.3e} px")
    assert err < 2e-3
    assert np.array_equal(valid.cpu().numpy().astype(bool), valid_o)


def test_bitwise_deterministic(dp, ctx):
    s = make_window(3)
    a = _gpu_solve(dp, ctx, s, dp.FP32)
    b = _gpu_solve(dp, ctx, s, dp.FP32)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp32", "fp64", "mixed"])
@pytest.mark.parametrize("scene", ["window", "blocked"])
def test_cooperative_launch_matches_ordinary(dp, ctx, prec, scene):
    # the single-launch solver (window) and the chained triangular solves of
    # the blocked factorisation (300 unknowns) give the same bits under either launch
    s = make_window(11) if scene == "window" else tiny_scene(52, 12, seed=4, radius=5, trajectory="forward")
    try:
        ctx.set_cooperative(True)
        a = _gpu_solve(dp, ctx, s, PREC[prec])
    finally:
        ctx.set_cooperative(False)
    b = _gpu_solve(dp, ctx, s, PREC[prec])
    assert a[2]["status"] == 0 and b[2]["status"] == 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2]["cost"] == b[2]["cost"]
    assert dp.binding.lib().dpvba_set_cooperative(ctx._h, 2) == dp.binding.DPVBA_EINVAL


def _edit(s: Scene, **kw) -> Scene:
    d = dict(s.__dict__)
    d.update(kw)
    return Scene(**d)


def test_edge_order_and_duplicates(dp, ctx):
    base = tiny_scene(5, 7, seed=9)
    rng = np.random.default_rng(0)
    perm = rng.permutation(base.n_edges)
    dup = np.concatenate([perm, perm[:5]])
    s = _edit(base, ii=base.ii[dup], jj=base.jj[dup], kk=base.kk[dup], target=base.target[dup],
              weight=base.weight[dup], target64=base.target64[dup])
    Po, Do, _ = ba64.solve_scene(s)
    P, D, rep = _gpu_solve(dp, ctx, s, dp.FP64)
    _compare(s, P, D, Po, Do, TOL["fp64"], "permuted+duplicated fp64")


def test_patches_without_edges_and_structure_only(dp, ctx):
    base = tiny_scene(5, 7, seed=10)
    keep = base.kk % 7 != 3   # patch 3 of every frame loses its edges
    s = _edit(base, ii=base.ii[keep], jj=base.jj[keep], kk=base.kk[keep], target=base.target[keep],
              weight=base.weight[keep], target64=base.target64[keep])
    Po, Do, _ = ba64.solve_scene(s)
    P, D, _ = _gpu_solve(dp, ctx, s, dp.FP64)
    _compare(s, P, D, Po, Do, TOL["fp64"], "edgeless patches fp64")
    assert np.array_equal(D[3::7], s.inv_depth[3::7].astype(np.float64))
    so = _edit(base, n_fixed=base.n_frames)
    Po, Do, _ = ba64.solve_scene(so)
    P, D, _ = _gpu_solve(dp, ctx, so, dp.FP64)
    _compare(so, P, D, Po, Do, TOL["fp64"], "structure-only fp64")


def test_batched_window_shapes(dp, ctx):
    # a few of the batched-workload instances, including the widest reduced system
    from scenes.patchgraph import instance_shapes
    shapes = instance_shapes(4, 256)
    widest = int(np.argmax([F for F, K, r, nf in shapes]))
    for b in (0, 1, widest):
        s = make_config(4, b)
        Po, Do, _ = ba64.solve_scene(s)
        P, D, rep = _gpu_solve(dp, ctx, s, dp.FP32)
        _compare(s, P, D, Po, Do, TOL["fp32"], f"{s.name} fp32")


def test_rejects_bad_graph(dp, ctx):
    s = tiny_scene(4, 5, seed=1)
    bad = _edit(s, jj=s.ii.copy())   # self edges
    with pytest.raises(dp.DpvbaError):
        ctx.analyze(dp.GraphTensors.from_scene(bad))
    kk = s.kk.copy(); kk[0] = s.n_patches   # out of range
    with pytest.raises(dp.DpvbaError):
        ctx.analyze(dp.GraphTensors.from_scene(_edit(s, kk=kk)))
    ii = s.ii.copy(); ii[0] = (ii[0] + 1) % s.n_frames   # patch owner inconsistent
    ii[0] = ii[0] if ii[0] != s.jj[0] else (ii[0] + 1) % s.n_frames
    with pytest.raises(dp.DpvbaError):
        ctx.analyze(dp.GraphTensors.from_scene(_edit(s, ii=ii)))


def _align_scale(P, Po):
    """Least-squares scale about pose 0 mapping P's camera centres onto Po's."""
    a = P[:, :3] - P[0, :3]
    b = Po[:, :3] - Po[0, :3]
    return float(np.sum(a * b) / np.sum(a * a))


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_global_ba_matches_oracle_golden(dp, ctx, prec):
    # 1000 keyframes, 1,505,568 edges, 5 iterations, n = 5994 (blocked path);
    # expected values written by tests/golden/make_global_ba_golden.py
    import os
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "global_ba_oracle.npz"))
    s = make_config(2)
    _log(f"global BA {prec}: E={s.n_edges}")
    P, D, rep = _gpu_solve(dp, ctx, s, PREC[prec])
    _log(f"  status {rep['status']} cost {rep['cost']} vs {list(gold['cost'])}")
    _log(f"  min pivot {rep['min_pivot']} refine {rep['refine_resid']} fallback {rep['fp64_fallback']}")
    assert rep["status"] == 0
    assert rep["n_invalid"] == list(gold["n_invalid"])
    dt, dr = ba64.pose_errors(P, gold["poses"])
    rel = np.abs(D - gold["inv_depth"]) / np.abs(gold["inv_depth"])
    sc = _align_scale(P, gold["poses"])
    Ps = P.copy(); Ps[:, :3] = P[0, :3] + sc * (P[:, :3] - P[0, :3])
    dts, _ = ba64.pose_errors(Ps, gold["poses"])
    _log(f"  raw: dt {dt.max():.3e} dr {dr.max():.3e} depth rel {rel.max():.3e}; "
         f"scale-aligned dt {dts.max():.3e} (scale {sc - 1:+.2e})")
    tol = TOL[prec]
    assert dr.max() < tol and dt.max() < tol and rel.max() < tol


def test_precisions_in_turn_after_one_analysis(dp, ctx):
    # one analysis, then float32, float64, mixed, float64, float32 solves on
    # the same context: the large path's reduced system buffer is shared by
    # the precisions (and only the envelope is gathered into it), so each
    # solve must start from a clean system whatever the previous one left
    from scenes import make_sweep
    s = make_sweep(200, total_patches=9600)
    Po, Do, _ = ba64.solve_scene(s)
    g = dp.GraphTensors.from_scene(s)
    ctx.analyze(g)
    for prec in ("fp32", "fp64", "mixed", "fp64", "fp32"):
        dt = torch.float64 if PREC[prec] == dp.FP64 else torch.float32
        poses = torch.as_tensor(s.poses, dtype=dt).cuda().contiguous()
        depth = torch.as_tensor(s.inv_depth, dtype=dt).cuda().contiguous()
        rep = ctx.solve(g, poses, depth, n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, precision=PREC[prec])
        assert rep["status"] == 0
        _compare(s, poses.double().cpu().numpy(), depth.double().cpu().numpy(), Po, Do, TOL[prec],
                 f"in turn {prec}")
