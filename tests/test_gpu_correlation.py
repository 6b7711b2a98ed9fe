"""Patch correlation of eq. 4 on the GPU (dpvba_patch_correlation) against
the float64 oracle (oracle/correlation.py).  The kernel accumulates float32
dot products of length D, so the bound per value is the dot-product bound
(D + 8) 2^-24 times the same correlation of |g| and |f|."""
import numpy as np
import pytest
import torch

from oracle import correlation

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


def _bound(g, f, kk, jj, xy):
    D = g.shape[-1]
    return (D + 8) * 2.0 ** -24 * correlation.correlation(np.abs(g), np.abs(f), kk, jj, xy) + 1e-30


def _run(ctx, g, f, kk, jj, xy):
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()
    return ctx.patch_correlation(t(g, torch.float32), t(f, torch.float32), t(kk, torch.int32), t(jj, torch.int32),
                                 t(xy, torch.float32)).cpu().numpy()


@pytest.mark.parametrize("D", [64, 128, 192, 256])
def test_random_points_and_borders(dp, ctx, D):
    rng = np.random.default_rng(D)
    E, p, M, H, W, P = 40, 3, 3, 20, 24, 7
    print(f"correlation D={D} E={E} map {H}x{W}", flush=True)
    g = rng.standard_normal((P, p, p, D)).astype(np.float32)
    f = rng.standard_normal((M, H, W, D)).astype(np.float32)
    kk = rng.integers(0, P, E)
    jj = rng.integers(0, M, E)
    xy = np.stack([rng.uniform(-6, W + 6, (E, p, p)), rng.uniform(-6, H + 6, (E, p, p))], -1).astype(np.float32)
    xy[0] = 5.0                                   # integer point
    xy[1, :, :, 0] = -0.5                         # half outside
    xy[2] = np.float32(1e20)                      # far outside
    xy[3, :, :, 1] = H - 1 + 0.25                 # bottom rows
    C = _run(ctx, g, f, kk, jj, xy)
    want = correlation.correlation(g, f, kk, jj, xy)
    bound = _bound(g, f, kk, jj, xy)
    err = np.abs(C - want)
    print(f"  max err {err.max():.3e}, worst err/bound {(err / bound).max():.3f}", flush=True)
    assert np.all(err <= bound)
    assert np.all(C[2] == 0.0)


def test_reprojected_window_patches(dp, ctx):
    """Coordinates from dpvba_reproject of a sliding window, at a quarter of
    the image resolution, against 22 feature maps of 120 x 160 x 128."""
    from scenes import make_window
    s = make_window(3)
    g_ = dp.GraphTensors.from_scene(s)
    poses = torch.as_tensor(s.poses).cuda()
    depth = torch.as_tensor(s.inv_depth).cuda()
    coords, _ = ctx.reproject(g_, poses, depth)
    xy = (coords / 4.0).contiguous()
    rng = np.random.default_rng(7)
    D, H, W = 128, 120, 160
    gm = torch.as_tensor(rng.standard_normal((s.n_patches, 3, 3, D)).astype(np.float32)).cuda()
    fm = torch.as_tensor(rng.standard_normal((s.n_frames, H, W, D)).astype(np.float32)).cuda()
    C = ctx.patch_correlation(gm, fm, g_.kk, g_.jj, xy).cpu().numpy()
    sample = rng.choice(s.n_edges, 150, replace=False)
    xs = xy.cpu().numpy()[sample]
    gn, fn = gm.cpu().numpy(), fm.cpu().numpy()
    want = correlation.correlation(gn, fn, s.kk[sample], s.jj[sample], xs)
    bound = _bound(gn, fn, s.kk[sample], s.jj[sample], xs)
    err = np.abs(C[sample] - want)
    print(f"window correlation: E={s.n_edges}, sampled max err {err.max():.3e}, err/bound {(err / bound).max():.3f}",
          flush=True)
    assert np.all(err <= bound)


def test_bad_index_is_reported(dp, ctx):
    rng = np.random.default_rng(1)
    g = rng.standard_normal((2, 1, 1, 64)).astype(np.float32)
    f = rng.standard_normal((1, 8, 8, 64)).astype(np.float32)
    xy = np.full((2, 1, 1, 2), 3.0, dtype=np.float32)
    C = _run(ctx, g, f, np.array([0, 5]), np.array([0, 0]), xy)
    assert np.all(C[1] == 0.0) and np.any(C[0] != 0.0)
    assert ctx.device_status() == (dp.binding.DPVBA_EDEVICE, 4)
    assert ctx.device_status() == (dp.binding.DPVBA_OK, 0)
