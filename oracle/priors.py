"""Network outputs at the network's resolution -> keyframe priors (Sec. II-A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network takes and returns 256 x 192 images: log-depth, its variance, the x
and y log-depth gradients and their variances. Its log-depths are normalised by
the focal length of the camera it was trained with; at test time they are scaled
by the focal length of the camera in use, which in log space is one added
constant, and the gradients and uncertainties need no such scaling (Sec. II-A,
last paragraphs). Readings (R25):
  - maps are resampled to the keyframe's W x H bilinearly with pixel centres
    aligned: keyframe pixel u samples the network map at
    u_n = (u + 1/2) W_n / W - 1/2, clamped to [0, W_n - 1] (likewise v);
  - the log-depth shift is ln(f_n / f_ref), with f_n = f_x W_n / W the keyframe
    camera's focal length in pixels at the network's resolution and f_ref the
    training camera's, in the same units;
  - the gradients are per network pixel; per keyframe pixel they scale by the
    spacing ratio (W_n / W for x, H_n / H for y) and their variances by its
    square. The log-depth variance is resampled unchanged.
"""

from __future__ import annotations

import numpy as np


def sample_positions(n_out: int, n_in: int) -> np.ndarray:
    """Network-map coordinates of the keyframe pixel centres along one axis."""
    u = (np.arange(n_out, dtype=np.float64) + 0.5) * (n_in / n_out) - 0.5
    return np.clip(u, 0.0, n_in - 1.0)


def resample_bilinear(img: np.ndarray, W: int, H: int) -> np.ndarray:
    """img (H_n x W_n) sampled at the keyframe pixel centres (H x W)."""
    img = np.asarray(img, dtype=np.float64)
    Hn, Wn = img.shape
    un = sample_positions(W, Wn)
    vn = sample_positions(H, Hn)
    u0 = np.minimum(np.floor(un), Wn - 2).astype(np.int64)
    v0 = np.minimum(np.floor(vn), Hn - 2).astype(np.int64)
    f = un - u0
    g = vn - v0
    out = np.empty((H, W))
    for r in range(H):
        a = img[v0[r]]
        b = img[v0[r] + 1]
        top = (1.0 - f) * a[u0] + f * a[u0 + 1]
        bot = (1.0 - f) * b[u0] + f * b[u0 + 1]
        out[r] = (1.0 - g[r]) * top + g[r] * bot
    return out


def network_priors(maps_net, W: int, H: int, fx: float, focal_ref: float):
    """(mu, var_mu, g_x, var_gx, g_y, var_gy) at keyframe resolution from the
    network's six maps at its own resolution."""
    mu_n, vmu_n, gx_n, vgx_n, gy_n, vgy_n = (np.asarray(m, dtype=np.float64) for m in maps_net)
    Hn, Wn = mu_n.shape
    sx, sy = Wn / W, Hn / H
    shift = np.log(fx * sx / focal_ref)
    mu = resample_bilinear(mu_n, W, H) + shift
    vmu = resample_bilinear(vmu_n, W, H)
    gx = resample_bilinear(gx_n, W, H) * sx
    vgx = resample_bilinear(vgx_n, W, H) * (sx * sx)
    gy = resample_bilinear(gy_n, W, H) * sy
    vgy = resample_bilinear(vgy_n, W, H) * (sy * sy)
    return mu, vmu, gx, vgx, gy, vgy
