"""Pose-error measures between two Sim(3) estimates (oracle; test infrastructure
only).

* rotation: the angle of R_a R_b^T, taken as atan2(|vee(M - M^T)|, tr M - 1),
  which keeps full precision near zero where acos would not
* scale: |s_a / s_b - 1|
* translation: |t_a - t_b| / max(|t_b|, 1 m)
"""

import numpy as np


def rotation_angle(Ra, Rb):
    M = np.asarray(Ra, dtype=np.float64) @ np.asarray(Rb, dtype=np.float64).T
    v = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    return float(np.arctan2(np.linalg.norm(v), np.trace(M) - 1.0))


def scale_error(sa, sb):
    return float(abs(sa / sb - 1.0))


def translation_error(ta, tb):
    ta = np.asarray(ta, dtype=np.float64)
    tb = np.asarray(tb, dtype=np.float64)
    return float(np.linalg.norm(ta - tb) / max(np.linalg.norm(tb), 1.0))


def pose_errors(a, b):
    """a, b: (s, R, t) triples. Returns (rotation rad, rel scale, rel translation)."""
    return (rotation_angle(a[1], b[1]), scale_error(a[0], b[0]),
            translation_error(a[2], b[2]))
