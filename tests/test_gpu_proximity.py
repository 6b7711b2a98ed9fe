"""Proximity loop-closure edges on the GPU (dpvba_proximity_edges) against
the oracle (oracle/proximity.py): integer results, compared exactly, on the
1000-keyframe workload's cameras (true and drifted), on cameras with exact
ties and on degenerate arguments; and the device-built graph of the global
BA (temporal plus loop edges) solves like the workload's own."""
import numpy as np
import pytest
import torch

from oracle import proximity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dp():
    import paper_2408_01654_amd as dp
    return dp


@pytest.fixture(scope="module")
def ctx(dp):
    c = dp.Context(0)
    yield c
    c.close()


def _check(ctx, poses, patch_off, first_recent, min_gap, radius, max_targets, what):
    print(f"proximity {what}: N={len(poses)} recent>={first_recent} gap {min_gap} r {radius} k {max_targets}",
          flush=True)
    P = torch.as_tensor(np.asarray(poses, dtype=np.float32)).cuda().contiguous()
    off = torch.as_tensor(np.asarray(patch_off, dtype=np.int32)).cuda().contiguous()
    counts, targets, edge_off, ii, jj, kk = ctx.proximity_edges(P, off, first_recent, min_gap, radius, max_targets)
    want = proximity.loop_targets(np.asarray(poses, dtype=np.float32)[:, :3], first_recent, min_gap, radius,
                                  max_targets)
    got_t = targets.cpu().numpy()
    assert counts.cpu().tolist() == [len(t) for t in want]
    for i, t in enumerate(want):
        assert got_t[i, :len(t)].tolist() == t and np.all(got_t[i, len(t):] == -1), i
    wi, wj, wk = proximity.loop_edges(want, np.asarray(patch_off))
    assert np.array_equal(ii.cpu().numpy(), wi) and np.array_equal(jj.cpu().numpy(), wj)
    assert np.array_equal(kk.cpu().numpy(), wk)
    eo = edge_off.cpu().numpy()
    assert eo[0] == 0 and eo[-1] == len(wi)
    return len(wi)


def test_global_workload_cameras(dp, ctx):
    from scenes import make_config
    s = make_config(2)
    off = np.arange(0, 96 * (s.n_frames + 1), 96)
    n_gt = _check(ctx, s.poses_gt.astype(np.float32), off, 0, 100, 2.0, 10, "ground truth")
    assert n_gt == 3725 * 96
    _check(ctx, s.poses, off, 0, 100, 2.0, 10, "drifted start")
    _check(ctx, s.poses, off, 900, 100, 2.0, 10, "recent frames only")
    _check(ctx, s.poses, off, 0, 50, 3.0, 32, "wide")


def test_ties_and_uneven_patches(dp, ctx):
    rng = np.random.default_rng(3)
    n = 300
    poses = np.zeros((n, 7), dtype=np.float32)
    poses[:, :3] = rng.integers(-3, 4, size=(n, 3)).astype(np.float32)   # many exact ties
    poses[:, 6] = 1.0
    off = np.concatenate([[0], np.cumsum(rng.integers(0, 9, size=n))])
    _check(ctx, poses, off, 0, 5, 2.0, 7, "integer grid")
    _check(ctx, poses, off, 100, 0, 1.5, 32, "integer grid, all gaps")


def test_degenerate_arguments(dp, ctx):
    poses = np.zeros((5, 7), dtype=np.float32)
    poses[:, 6] = 1.0
    off = np.arange(0, 6 * 3, 3)
    assert _check(ctx, poses, off, 0, 0, 1.0, 0, "no targets") == 0
    assert _check(ctx, poses, off, 5, 0, 1.0, 4, "no recent frame") == 0
    assert _check(ctx, poses, off, 0, 0, 0.0, 4, "empty radius") == 0
    assert _check(ctx, poses, off, 0, 9, 1.0, 4, "gap beyond") == 0
    assert _check(ctx, poses, off, 0, 0, 1.0, 4, "all together") == 3 * (4 + 3 + 2 + 1)
    with pytest.raises(dp.DpvbaError):
        ctx.proximity_edges(torch.as_tensor(poses).cuda(), torch.as_tensor(off.astype(np.int32)).cuda(), 0, 0, 1.0,
                            33)


def test_device_graph_solves_like_the_workload(dp, ctx):
    """Temporal edges of the workload plus the loop edges built on the device
    from the true cameras: the same edge multiset as the workload, so one
    solve of the reordered graph agrees with the stored oracle result."""
    import os
    from oracle import ba64
    from scenes import make_config
    s = make_config(2)
    off = torch.arange(0, 96 * (s.n_frames + 1), 96, dtype=torch.int32).cuda()
    _, _, _, ii, jj, kk = ctx.proximity_edges(torch.as_tensor(s.poses_gt.astype(np.float32)).cuda(), off, 0, 100,
                                              2.0, 10)
    temporal = np.abs(s.jj.astype(np.int64) - s.ii) <= 6
    key_w = {(int(a), int(b), int(c)): e for e, (a, b, c) in enumerate(zip(s.ii, s.jj, s.kk))}
    loop_idx = np.array([key_w[(int(a), int(b), int(c))] for a, b, c in
                         zip(ii.cpu().numpy(), jj.cpu().numpy(), kk.cpu().numpy())])
    order = np.concatenate([np.flatnonzero(temporal), loop_idx])
    assert np.array_equal(np.sort(order), np.arange(s.n_edges))
    g = dp.GraphTensors(s.n_frames, s.n_fixed, torch.as_tensor(s.patches).cuda(),
                        torch.as_tensor(s.ii[order]).cuda(), torch.as_tensor(s.jj[order]).cuda(),
                        torch.as_tensor(s.kk[order]).cuda(), torch.as_tensor(s.target[order]).cuda(),
                        torch.as_tensor(s.weight[order]).cuda(), tuple(float(x) for x in s.intrinsics))
    ctx.analyze(g)
    poses = torch.as_tensor(s.poses).cuda().contiguous()
    depth = torch.as_tensor(s.inv_depth).cuda().contiguous()
    rep = ctx.solve(g, poses, depth, n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, precision=dp.FP32)
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "global_ba_oracle.npz"))
    dt, dr = ba64.pose_errors(poses.double().cpu().numpy(), gold["poses"])
    rel = np.abs(depth.double().cpu().numpy() - gold["inv_depth"]) / np.abs(gold["inv_depth"])
    print(f"device-built graph: status {rep['status']} dt {dt.max():.2e} dr {dr.max():.2e} depth {rel.max():.2e}",
          flush=True)
    assert rep["status"] == 0 and max(dt.max(), dr.max(), rel.max()) < 1e-4
