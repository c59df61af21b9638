"""Pins of the pose-error measures (oracle/metrics.py) that every parity check
uses: the angle of the relative rotation, the relative scale error and the
relative translation error with its 1 m floor.

Each is checked against values fixed independently of its formula: rotations
built from an axis and an angle by scipy (the angle is known), scipy's own
quaternion-based magnitude of the relative rotation, group invariances, and
hand-computed scale and translation cases. A dropped transpose, a wrong sign
in the trace term, a missing absolute value or a wrong floor each fails one of
them."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import metrics


@pytest.mark.parametrize("theta", [1e-9, 1e-4, 0.5, 3.0, np.pi - 1e-6])
def test_rotation_angle_of_axis_angle(theta):
    rng = np.random.default_rng(11)
    for _ in range(5):
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        R = Rotation.from_rotvec(theta * a).as_matrix()
        got = metrics.rotation_angle(R, np.eye(3))
        # relative precision near 0, absolute precision elsewhere
        assert abs(got - theta) <= 1e-12 * theta + 1e-14, (theta, got)
        assert abs(metrics.rotation_angle(np.eye(3), R) - theta) <= 1e-12 * theta + 1e-14


def test_rotation_angle_matches_scipy_magnitude():
    rng = np.random.default_rng(12)
    Ra = Rotation.random(200, random_state=rng)
    Rb = Rotation.random(200, random_state=rng)
    for a, b in zip(Ra, Rb):
        ref = (a * b.inv()).magnitude()      # quaternion route, independent of the trace form
        got = metrics.rotation_angle(a.as_matrix(), b.as_matrix())
        assert abs(got - ref) <= 1e-9, (got, ref)


def test_rotation_angle_zero_and_invariances():
    rng = np.random.default_rng(13)
    for _ in range(20):
        R = Rotation.random(random_state=rng).as_matrix()
        G = Rotation.random(random_state=rng).as_matrix()
        R2 = Rotation.random(random_state=rng).as_matrix()
        # a rotation against itself: zero (fails if the transpose is dropped)
        assert metrics.rotation_angle(R, R) <= 1e-7
        th = metrics.rotation_angle(R, R2)
        # left and right invariance of the relative angle
        assert abs(metrics.rotation_angle(G @ R, G @ R2) - th) <= 1e-9
        assert abs(metrics.rotation_angle(R @ G, R2 @ G) - th) <= 1e-9
        assert 0.0 <= th <= np.pi


def test_rotation_angle_small_relative_perturbation():
    # a known 1e-7 rad perturbation of a generic rotation is reported as such:
    # the measure resolves errors far below the 1e-5 rad parity tolerance
    rng = np.random.default_rng(14)
    R = Rotation.random(random_state=rng).as_matrix()
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    for eps in (1e-7, 1e-6, 1e-5):
        Rp = Rotation.from_rotvec(eps * a).as_matrix() @ R
        assert abs(metrics.rotation_angle(Rp, R) - eps) <= 1e-3 * eps


def test_scale_error_hand_computed():
    assert metrics.scale_error(1.1, 1.0) == pytest.approx(0.1, rel=1e-12)
    assert metrics.scale_error(0.9, 1.0) == pytest.approx(0.1, rel=1e-12)     # sign dropped
    assert metrics.scale_error(2.0, 4.0) == pytest.approx(0.5, rel=1e-12)     # relative to the second
    assert metrics.scale_error(4.0, 2.0) == pytest.approx(1.0, rel=1e-12)
    assert metrics.scale_error(3.0, 3.0) == 0.0


def test_translation_error_hand_computed():
    # below 1 m the denominator is the 1 m floor
    assert metrics.translation_error([0.5, 0.0, 0.0], [0.0, 0.0, 0.0]) == pytest.approx(0.5, rel=1e-12)
    assert metrics.translation_error([0.0, 0.3, 0.4], [0.0, 0.0, 0.2]) == pytest.approx(np.hypot(0.3, 0.2),
                                                                                       rel=1e-12)
    # above 1 m it is relative to the second argument's length
    assert metrics.translation_error([3.0, 0.0, 0.0], [2.0, 0.0, 0.0]) == pytest.approx(0.5, rel=1e-12)
    assert metrics.translation_error([2.0, 0.0, 0.0], [3.0, 0.0, 0.0]) == pytest.approx(1.0 / 3.0, rel=1e-12)
    # Euclidean length of the difference: |(1, 2, 2)| = 3 over |(0, 0, 6)| = 6
    assert metrics.translation_error([1.0, 2.0, 8.0], [0.0, 0.0, 6.0]) == pytest.approx(0.5, rel=1e-12)
    assert metrics.translation_error([-1.0, -2.0, 4.0], [0.0, 0.0, 6.0]) == pytest.approx(0.5, rel=1e-12)


def test_pose_errors_order_and_components():
    Ra = Rotation.from_rotvec([0.0, 0.0, 0.25]).as_matrix()
    a = (1.5, Ra, np.array([4.0, 0.0, 0.0]))
    b = (1.0, np.eye(3), np.array([0.0, 0.0, 2.0]))
    rot, sc, tr = metrics.pose_errors(a, b)
    assert rot == pytest.approx(0.25, rel=1e-12)
    assert sc == pytest.approx(0.5, rel=1e-12)
    assert tr == pytest.approx(np.hypot(4.0, 2.0) / 2.0, rel=1e-12)
