"""Pins for the gradient oracle (oracle/grad64.py): its forward agrees with
the independent numpy oracle, and its reverse-mode gradients with respect to
targets and weights agree with central finite differences of the loss."""
import numpy as np
import pytest

from oracle import ba64, grad64, lie64
from scenes import tiny_scene, make_config


@pytest.mark.parametrize("mk", [lambda: tiny_scene(5, 6, seed=31), lambda: tiny_scene(6, 5, seed=32, radius=2)])
def test_forward_matches_numpy_oracle(mk):
    s = mk()
    P, D, _ = ba64.solve_scene(s)
    R, t, d = grad64.forward_state(s)
    Ro, to = lie64.pose_to_rt(P)
    np.testing.assert_allclose(R, Ro, atol=1e-12)
    np.testing.assert_allclose(t, to, atol=1e-12)
    np.testing.assert_allclose(d, D, rtol=1e-11)


def test_forward_matches_on_a_window():
    s = make_config(3, 0)
    P, D, _ = ba64.solve_scene(s)
    R, t, d = grad64.forward_state(s)
    Ro, to = lie64.pose_to_rt(P)
    np.testing.assert_allclose(R, Ro, atol=1e-11)
    np.testing.assert_allclose(t, to, atol=1e-11)
    np.testing.assert_allclose(d, D, rtol=1e-10)


@pytest.mark.parametrize("seed", [41, 42])
def test_gradients_match_central_differences(seed):
    s = tiny_scene(5, 5, seed=seed)
    L, gt, gw = grad64.loss_and_grads(s)
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
