"""Pins of the patch-correlation oracle (oracle/correlation.py, eq. 4): the
integer-coordinate closed form (plain indexing), scipy's linear
interpolation, exact interpolation of a linear map, and hand-worked border
values."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import correlation


def _inputs(seed, E=6, p=3, D=8, M=3, H=11, W=14):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((5, p, p, D)).astype(np.float32)
    f = rng.standard_normal((M, H, W, D)).astype(np.float32)
    kk = rng.integers(0, 5, E)
    jj = rng.integers(0, M, E)
    return g, f, kk, jj, rng


def test_integer_points_index_the_map():
    g, f, kk, jj, rng = _inputs(0)
    E, p, H, W = 6, 3, f.shape[1], f.shape[2]
    xy = np.stack([rng.integers(-2, W + 2, (E, p, p)), rng.integers(-2, H + 2, (E, p, p))], -1).astype(np.float32)
    C = correlation.correlation(g, f, kk, jj, xy)
    for e in range(E):
        for u in range(p):
            for v in range(p):
                for a in range(7):
                    for b in range(7):
                        x, y = int(xy[e, u, v, 0]) + a - 3, int(xy[e, u, v, 1]) + b - 3
                        want = 0.0
                        if 0 <= x < W and 0 <= y < H:
                            want = float(np.dot(g[kk[e], u, v].astype(np.float64), f[jj[e], y, x]))
                        assert C[e, u, v, a, b] == pytest.approx(want, abs=1e-12)


def test_matches_scipy_linear_interpolation():
    g, f, kk, jj, rng = _inputs(1)
    E, p, H, W, D = 6, 3, f.shape[1], f.shape[2], f.shape[3]
    # interior points: the 7 x 7 grid stays 1 pixel away from the border
    xy = np.stack([rng.uniform(4, W - 5, (E, p, p)), rng.uniform(4, H - 5, (E, p, p))], -1).astype(np.float32)
    C = correlation.correlation(g, f, kk, jj, xy)
    off = np.arange(7) - 3
    for e in range(E):
        for u in range(p):
            for v in range(p):
                X = xy[e, u, v, 0] + off[:, None] + 0 * off[None, :]
                Y = xy[e, u, v, 1] + 0 * off[:, None] + off[None, :]
                samp = np.stack([ndimage.map_coordinates(f[jj[e], :, :, d].astype(np.float64), [Y, X], order=1,
                                                         mode="nearest") for d in range(D)], -1)
                want = samp @ g[kk[e], u, v].astype(np.float64)
                np.testing.assert_allclose(C[e, u, v], want, rtol=1e-10, atol=1e-10)


def test_linear_map_is_reproduced_exactly():
    H, W, D = 12, 15, 4
    coef = np.array([[0.5, -1.25, 2.0], [1.0, 0.25, -0.5], [-0.75, 0.5, 1.5], [0.0, 2.0, 0.25]])  # [D, (a, b, c)]
    yy, xx = np.mgrid[0:H, 0:W]
    f = np.stack([c[0] * xx + c[1] * yy + c[2] for c in coef], -1)[None].astype(np.float32)
    g = np.array([[[[1.0, -2.0, 0.5, 3.0]]]], dtype=np.float32)
    xy = np.array([[[[6.3, 5.7]]]], dtype=np.float32)
    C = correlation.correlation(g, f, [0], [0], xy)
    off = np.arange(7) - 3
    for a in range(7):
        for b in range(7):
            x, y = float(xy[0, 0, 0, 0]) + off[a], float(xy[0, 0, 0, 1]) + off[b]
            want = sum(float(g[0, 0, 0, d]) * (coef[d, 0] * x + coef[d, 1] * y + coef[d, 2]) for d in range(D))
            assert C[0, 0, 0, a, b] == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_border_weights():
    f = np.ones((1, 4, 4, 1), dtype=np.float32)
    g = np.ones((1, 1, 1, 1), dtype=np.float32)
    # centre of the grid at (-0.5 + 3, 1): offset a = 0 puts the point at x = -0.5,
    # half of its weight on the missing column x = -1
    xy = np.array([[[[2.5, 1.0]]]], dtype=np.float32)
    C = correlation.correlation(g, f, [0], [0], xy)[0, 0, 0]
    assert C[0, 3] == pytest.approx(0.5)   # x = -0.5
    assert C[1, 3] == pytest.approx(1.0)   # x = 0.5
    assert C[4, 3] == pytest.approx(0.5)   # x = 3.5
    assert C[6, 3] == pytest.approx(0.0)   # x = 5.5
    assert C[3, 0] == pytest.approx(0.0)   # y = -2
    assert C[3, 2] == pytest.approx(1.0)   # y = 0
    assert C[0, 0] == pytest.approx(0.0)
