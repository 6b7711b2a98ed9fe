"""Seeded scene generator: sizes of the workloads, determinism, ordering."""
import numpy as np
import pytest

from scenes import make_config, make_window, tiny_scene
from scenes.patchgraph import instance_shapes


def test_cfg0_shape():
    s = make_config(0)
    assert (s.n_frames, s.n_patches, s.n_edges, s.n_fixed) == (8, 768, 5376, 2)


def test_window_shape_and_shared_structure():
    a, b = make_window(0), make_window(17)
    assert (a.n_frames, a.n_patches, a.n_edges, a.n_fixed) == (22, 2112, 37440, 10)
    for f in ("ii", "jj", "kk"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert not np.array_equal(a.target, b.target)


@pytest.mark.slow
def test_cfg2_shape():
    s = make_config(2)
    assert (s.n_frames, s.n_patches, s.n_edges, s.n_fixed) == (1000, 96000, 1505568, 1)
    assert s.meta["loop_pairs"] == 3725


def test_determinism_and_order():
    a, b = make_config(0), make_config(0)
    for f in ("poses", "patches", "inv_depth", "target", "weight"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    key = a.ii.astype(np.int64) * 10**12 + a.kk.astype(np.int64) * 10**4 + a.jj
    assert np.all(np.diff(key) > 0)
    # patch ownership: every edge of patch k leaves the same frame
    owner = np.full(a.n_patches, -1)
    owner[a.kk] = a.ii
    assert np.all(owner[a.kk] == a.ii)


def test_batched_instance_ranges():
    s3 = instance_shapes(3, 16)
    assert all(12 <= F <= 22 and 64 <= K <= 96 and nf == max(2, F - 12) for F, K, r, nf in s3)
    s4 = instance_shapes(4, 256)
    assert all(8 <= F <= 40 and 48 <= K <= 128 and 4 <= r <= 13 for F, K, r, nf in s4)


def test_generated_depths_positive_in_all_targets():
    s = tiny_scene(6, 10, seed=5, noise_px=0.0)
    assert np.all(s.inv_depth_gt > 0)
    assert np.all((s.weight > 0.1) & (s.weight <= 1.0))
