"""Pins of the proximity loop-closure oracle (oracle/proximity.py): a
hand-worked example (strict radius, gap, truncation to the nearest, ties to
the lower frame), a float64 brute force on random cameras, the edge layout,
and the loop edges of the 1000-keyframe global-BA workload."""
import math

import numpy as np
import pytest

from oracle import proximity


def _line(xs):
    return np.array([[x, 0.0, 0.0] for x in xs], dtype=np.float32)


def test_hand_worked_line():
    # cameras on the x axis; old frames need j - i > 2, loops closer than 1
    c = _line([0.0, 1.0, 2.0, 3.0, 0.5, 2.5, 0.0, 5.0])
    t = proximity.loop_targets(c, first_recent=0, min_gap=2, radius=1.0, max_targets=2)
    # frame 0: j = 4 (0.25) and j = 6 (0.0); frame 1: j = 4 (0.25), j = 6 lies at
    # exactly the radius (d^2 = 1 = r^2, excluded); frame 2: j = 5 (0.25)
    assert t == [[4, 6], [4], [5], [], [], [], [], []]
    # one target only: the nearest (frame 0 -> 6 at distance 0)
    t1 = proximity.loop_targets(c, first_recent=0, min_gap=2, radius=1.0, max_targets=1)
    assert t1[0] == [6] and t1[1] == [4]
    # recent frames only: j >= 6 leaves frame 0 -> 6 and nothing for frame 1 (d^2 = 1)
    t2 = proximity.loop_targets(c, first_recent=6, min_gap=2, radius=1.0, max_targets=2)
    assert t2 == [[6], [], [], [], [], [], [], []]


def test_tie_goes_to_lower_frame():
    c = _line([0.0, 9.0, 9.0, 0.5, -0.5, 0.25])
    t = proximity.loop_targets(c, first_recent=0, min_gap=2, radius=1.0, max_targets=1)
    assert t[0] == [5]          # 0.25 is nearest
    t = proximity.loop_targets(_line([0.0, 9.0, 9.0, 0.5, -0.5]), 0, 2, 1.0, 1)
    assert t[0] == [3]          # 0.5 and -0.5 tie: the lower frame
    t = proximity.loop_targets(_line([0.0, 9.0, 9.0, 0.5, -0.5]), 0, 2, 1.0, 2)
    assert t[0] == [3, 4]


def test_degenerate_arguments():
    c = _line([0.0, 0.0, 0.0])
    assert proximity.loop_targets(c, 0, 0, 1.0, 0) == [[], [], []]      # no targets allowed
    assert proximity.loop_targets(c, 0, 5, 1.0, 4) == [[], [], []]      # gap longer than the sequence
    assert proximity.loop_targets(c, 0, 0, 0.0, 4) == [[], [], []]      # empty radius (strict)
    assert proximity.loop_targets(c, 3, 0, 1.0, 4) == [[], [], []]      # no recent frame
    assert proximity.loop_targets(c, 0, 0, 1.0, 4) == [[1, 2], [2], []]


def _brute(c64, first_recent, min_gap, radius, max_targets):
    out = []
    for i in range(len(c64)):
        cand = []
        for j in range(len(c64)):
            if j - i > min_gap and j >= first_recent:
                d = math.dist(c64[i], c64[j])
                if d < radius:
                    cand.append((d, j))
        cand.sort()
        out.append(sorted(j for _, j in cand[:max_targets]))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_float64_brute_force(seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-3, 3, size=(120, 3)).astype(np.float32)
    c64 = c.astype(np.float64)
    r = 1.7
    # no pair lies so close to the radius that float32 rounding could flip it
    d = np.linalg.norm(c64[:, None] - c64[None], axis=-1)
    assert np.abs(d - r).min() > 1e-4
    got = proximity.loop_targets(c, first_recent=10, min_gap=7, radius=r, max_targets=5)
    assert got == _brute(c64, 10, 7, r, 5)


def test_edge_layout():
    t = [[3, 5], [], [4], [], [], []]
    off = np.array([0, 2, 5, 6, 9, 9, 12])
    ii, jj, kk = proximity.loop_edges(t, off)
    assert ii.tolist() == [0, 0, 0, 0, 2]
    assert kk.tolist() == [0, 0, 1, 1, 5]
    assert jj.tolist() == [3, 5, 3, 5, 4]


def test_global_ba_workload_loops():
    """Applied to the ground-truth cameras of the 1000-keyframe workload, the
    rule gives exactly that workload's loop edges (its edges beyond the +-6
    temporal neighbours), which its generator chose in float64."""
    from scenes import make_config
    s = make_config(2)
    t = proximity.loop_targets(s.poses_gt[:, :3].astype(np.float32), first_recent=0, min_gap=100, radius=2.0,
                               max_targets=10)
    off = np.arange(0, 96 * (s.n_frames + 1), 96)
    ii, jj, kk = proximity.loop_edges(t, off)
    loop = np.abs(s.jj.astype(np.int64) - s.ii) > 6
    want = np.stack([s.ii[loop], s.jj[loop], s.kk[loop]], 1)
    got = np.stack([ii, jj, kk], 1)
    assert got.shape == want.shape == (3725 * 96, 3)
    assert np.array_equal(got[np.lexsort(got.T[::-1])], want[np.lexsort(want.T[::-1])])
