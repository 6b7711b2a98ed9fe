"""FP64 CPU oracle for patch-graph Gauss-Newton bundle adjustment.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library and imports
nothing from it; both sides read the same seeded inputs from ``scenes``.

Contents
--------
lie64   SO(3)/SE(3) maps and quaternion conversions (float64).
ba64    reprojection (eq. 2), residuals and Jacobians, normal equations of the
        confidence-weighted objective (eq. 3), depth elimination by Schur
        complement, Cholesky solve of the reduced camera system, SE(3)
        retraction, and the fixed-count Gauss-Newton loop.
grad64  float64 autograd statement of the same unrolled iterations, used as
        the gradient oracle for the adjoint.

Every function here is pinned by CPU tests against closed forms, finite
differences, library routines and invariants; see tests/test_oracle_*.py.
"""
