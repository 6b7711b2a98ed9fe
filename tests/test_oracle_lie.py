"""Pins for the oracle's SO(3)/SE(3) helpers against library routines and
closed forms (matrix exponential of the twist, scipy rotations)."""
import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import lie64


def _twist(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = lie64.hat(xi[3:])
    M[:3, 3] = xi[:3]
    return M


@pytest.mark.parametrize("scale", [1e-9, 1e-4, 0.3, 2.0, 3.0])
def test_so3_exp_matches_scipy(scale):
    rng = np.random.default_rng(1)
    phi = scale * rng.normal(size=(20, 3))
    np.testing.assert_allclose(lie64.so3_exp(phi), Rotation.from_rotvec(phi).as_matrix(), atol=1e-14)


@pytest.mark.parametrize("scale", [1e-9, 1e-4, 0.3, 2.0])
def test_se3_exp_matches_matrix_exponential(scale):
    rng = np.random.default_rng(2)
    for _ in range(10):
        xi = scale * rng.normal(size=6)
        R, t = lie64.se3_exp(xi)
        T = scipy.linalg.expm(_twist(xi))
        np.testing.assert_allclose(R, T[:3, :3], atol=1e-13)
        np.testing.assert_allclose(t, T[:3, 3], atol=1e-13)


def test_quaternion_conversions_match_scipy():
    rng = np.random.default_rng(3)
    q = rng.normal(size=(50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    np.testing.assert_allclose(lie64.quat_to_rot(q), Rotation.from_quat(q).as_matrix(), atol=1e-14)
    R = Rotation.from_quat(q).as_matrix()
    q2 = lie64.rot_to_quat(R)
    q_ref = Rotation.from_matrix(R).as_quat()
    q_ref *= np.sign(q_ref[:, 3:4])
    np.testing.assert_allclose(q2, q_ref, atol=1e-14)


def test_so3_log_inverts_exp():
    rng = np.random.default_rng(4)
    for scale in (1e-8, 1e-3, 0.5, 2.5):
        phi = scale * rng.normal(size=(30, 3))
        phi = phi[np.linalg.norm(phi, axis=1) < np.pi - 1e-3]
        np.testing.assert_allclose(lie64.so3_log(lie64.so3_exp(phi)), phi, atol=1e-13)
    np.testing.assert_allclose(lie64.so3_log(Rotation.from_rotvec([[0, 0, np.pi - 1e-7]]).as_matrix()),
                               [[0, 0, np.pi - 1e-7]], atol=1e-6)


def test_right_retraction_is_group_product():
    rng = np.random.default_rng(5)
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t = rng.normal(size=3)
    xi = 0.2 * rng.normal(size=6)
    Rn, tn = lie64.retract_right(R, t, xi)
    G = np.eye(4); G[:3, :3] = R; G[:3, 3] = t
    Gn = G @ scipy.linalg.expm(_twist(xi))
    np.testing.assert_allclose(Rn, Gn[:3, :3], atol=1e-13)
    np.testing.assert_allclose(tn, Gn[:3, 3], atol=1e-13)
