"""Seeded synthetic patch-graph scenes shared by the GPU path and the oracle.

This package is a world simulator only: it places cameras on a trajectory,
draws patch centres and inverse depths, renders the resulting world points into
target cameras and adds pixel noise.  It holds none of the bundle-adjustment
arithmetic (no relative-pose transfer in inverse-depth form, no Jacobians,
normal equations, factorisations or retractions), so neither side can inherit a
mistake from the other through it.
"""
from .patchgraph import (  # noqa: F401
    FX, FY, CX, CY, IMG_W, IMG_H, PATCH,
    Scene, make_config, make_sweep, make_window, relabel_frames, tiny_scene, window_sequence,
    CONFIG_NAMES,
)
