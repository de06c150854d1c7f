"""Camera geometry of the photometric error (Sec. II-B).

The error of keyframe pixel x_i at depth d compares I_1 at
pi(K T_WC1^-1 T_WC0 rho(x_i, d)) with I_0(x_i), where rho back-projects the pixel
to the 3-D point d K^-1 (u, v, 1) (z-depth) and pi divides by the third
coordinate. Writing [R | t] = T_WC1^-1 T_WC0 and rho = 1/d (inverse depth):

    K (R d K^-1 x~ + t) = d (K R K^-1 x~ + rho K t)

so the projection is pi(A + rho b) with A = H x~, H = K R K^-1 and b = K t.
"""

from __future__ import annotations

import numpy as np


def relative_pose(T_wc0: np.ndarray, T_wc1: np.ndarray):
    """[R | t] mapping keyframe-camera coordinates to new-frame coordinates."""
    T = np.linalg.inv(np.asarray(T_wc1, dtype=np.float64)) @ np.asarray(T_wc0, dtype=np.float64)
    return T[:3, :3].copy(), T[:3, 3].copy()


def epipolar_constants(K: np.ndarray, T_wc0: np.ndarray, T_wc1: np.ndarray):
    """(H, b, e0): infinite homography K R K^-1, K t, and the keyframe epipole K c1.

    c1 = -R^T t is the new camera's centre in keyframe coordinates; its image
    K c1 (homogeneous) is where every keyframe epipolar line passes.
    """
    K = np.asarray(K, dtype=np.float64)
    R, t = relative_pose(T_wc0, T_wc1)
    Hinf = K @ R @ np.linalg.inv(K)
    b = K @ t
    e0 = K @ (-R.T @ t)
    return Hinf, b, e0


def project_through(Hinf, b, u, v, rho):
    """pi(H (u, v, 1) + rho b): image-1 position of keyframe pixel (u, v) at inverse depth rho.

    Also returns the third homogeneous coordinate (positive in front of camera 1).
    """
    X0 = Hinf[0, 0] * u + Hinf[0, 1] * v + Hinf[0, 2] + rho * b[0]
    X1 = Hinf[1, 0] * u + Hinf[1, 1] * v + Hinf[1, 2] + rho * b[1]
    X2 = Hinf[2, 0] * u + Hinf[2, 1] * v + Hinf[2, 2] + rho * b[2]
    return X0 / X2, X1 / X2, X2


def project_point(K, T_wc0, T_wc1, u, v, depth):
    """Reference chain of the paper's formula: back-project, transform, project.

    Used only to check ``project_through`` (the two routes must agree).
    """
    K = np.asarray(K, dtype=np.float64)
    Kinv = np.linalg.inv(K)
    ray = Kinv @ np.array([u, v, 1.0])
    X0 = np.append(depth * ray, 1.0)
    X1 = np.linalg.inv(T_wc1) @ T_wc0 @ X0
    p = K @ X1[:3]
    return p[0] / p[2], p[1] / p[2]
