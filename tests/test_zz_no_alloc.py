"""dpvba_solve_noalloc (per-call buffers in the library's static device
array) against dpvba_solve on the same inputs, through the C ABI: two calls
in a row, the second on a smaller problem, so the second call runs over the
first call's leftovers in the shared array.  Both entry points run the same
kernels in the same order, so the results must agree bit for bit; both are
also checked against the float64 oracle at the workload tolerances
(float32 1e-4, float64 1e-9: pose translation, rotation angle, relative
inverse depth)."""
import numpy as np
import pytest
import torch

from oracle import ba64
from scenes import make_window, tiny_scene

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "fp64": 1e-9}


@pytest.fixture(scope="module")
def dp():
    import paper_2408_01654_amd as dp
    return dp


def _run(dp, ctx, g, s, precision, noalloc):
    dt = torch.float64 if precision == dp.FP64 else torch.float32
    poses = torch.as_tensor(s.poses, dtype=dt).cuda().contiguous()
    depth = torch.as_tensor(s.inv_depth, dtype=dt).cuda().contiguous()
    rep = ctx.solve(g, poses, depth, n_iters=s.n_iters, lam=s.lam, z_min=s.z_min, precision=precision,
                    noalloc=noalloc)
    return poses.cpu(), depth.cpu(), rep


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_solve_on_two_calls(dp, prec):
    precision = dp.FP32 if prec == "fp32" else dp.FP64
    ctx = dp.Context(0)
    try:
        # a full 22-frame window, then a smaller 10-frame all-pairs problem
        for s in (make_window(11), tiny_scene(10, 32, seed=1)):
            print(f"noalloc {prec}: {s.name} N={s.n_frames} P={s.n_patches} E={s.n_edges}", flush=True)
            g = dp.GraphTensors.from_scene(s)
            ctx.analyze(g)
            Pn, Dn, rn = _run(dp, ctx, g, s, precision, noalloc=True)
            Pr, Dr, rr = _run(dp, ctx, g, s, precision, noalloc=False)
            assert rn["status"] == 0 and rr["status"] == 0
            assert torch.equal(Pn, Pr) and torch.equal(Dn, Dr)
            assert rn["cost"] == rr["cost"] and rn["min_pivot"] == rr["min_pivot"]
            Po, Do, _ = ba64.solve_scene(s)
            dt_, dr_ = ba64.pose_errors(Pn.double().numpy(), Po)
            rel = np.abs(Dn.double().numpy() - Do) / np.abs(Do)
            print(f"  vs oracle: dt {dt_.max():.2e} dr {dr_.max():.2e} depth rel {rel.max():.2e}", flush=True)
            assert max(dt_.max(), dr_.max(), rel.max()) < TOL[prec]
    finally:
        ctx.close()


def test_noalloc_limits(dp):
    ctx = dp.Context(0)
    try:
        s = tiny_scene(20, 8, seed=2, radius=4, trajectory="forward")   # 18 free poses: 109 unknowns
        g = dp.GraphTensors.from_scene(s)
        ctx.analyze(g)
        poses = torch.as_tensor(s.poses).cuda().contiguous()
        depth = torch.as_tensor(s.inv_depth).cuda().contiguous()
        with pytest.raises(dp.DpvbaError) as ei:
            ctx.solve(g, poses, depth, n_iters=2, precision=dp.FP32, noalloc=True)
        assert ei.value.status == dp.binding.DPVBA_ELIMIT
        with pytest.raises(dp.DpvbaError) as ei:
            ctx.solve(g, poses, depth, n_iters=2, precision=dp.MIXED, noalloc=True)
        assert ei.value.status == dp.binding.DPVBA_EINVAL
    finally:
        ctx.close()
