"""Pins of the network-output ingestion (Sec. II-A; reading R25): resampling to the
keyframe size with pixel centres aligned, the focal-length log-depth shift and the
spacing scale of the gradients."""

import numpy as np

from oracle.priors import network_priors, resample_bilinear, sample_positions


def _maps(Hn, Wn, seed=0):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(Hn, Wn)) if k % 2 == 0 else rng.uniform(0.01, 0.1, (Hn, Wn)) for k in range(6)]


def test_same_size_and_focal_is_the_identity():
    m = _maps(12, 16)
    out = network_priors(m, 16, 12, fx=300.0, focal_ref=300.0)
    for a, b in zip(m, out):
        assert np.array_equal(a, b)


def test_pixel_centres_are_aligned_by_hand():
    """2 x 2 -> 4 x 4: keyframe centres 0.5, 1.5, 2.5, 3.5 map to network
    coordinates -0.25, 0.25, 0.75, 1.25, clamped to 0, 0.25, 0.75, 1 (an
    unaligned u_n = u W_n / W would give 0, 0.5, 1, 1)."""
    assert np.allclose(sample_positions(4, 2), [0.0, 0.25, 0.75, 1.0])
    img = np.array([[0.0, 4.0], [8.0, 12.0]])
    out = resample_bilinear(img, 4, 4)
    assert np.allclose(out[0], [0.0, 1.0, 3.0, 4.0])
    assert np.allclose(out[:, 0], [0.0, 2.0, 6.0, 8.0])
    # halving: each keyframe pixel sits half way between two network pixels
    assert np.allclose(sample_positions(3, 6), [0.5, 2.5, 4.5])


def test_affine_fields_are_reproduced_and_gradients_match_finite_differences():
    """A log-depth plane a + b u_n + c v_n at 256 x 192 with its constant
    gradients (b, c) per network pixel: away from the clamped border the
    resampled log-depth is the same plane at the keyframe's sample positions, and
    its forward differences per keyframe pixel equal the resampled, rescaled
    gradient maps (b W_n / W, c H_n / H). A missing or inverted spacing factor
    fails."""
    Wn, Hn, W, H = 256, 192, 640, 480
    a, b, c = 0.7, 0.013, -0.008
    vv, uu = np.mgrid[0:Hn, 0:Wn].astype(np.float64)
    mu_n = a + b * uu + c * vv
    m = [mu_n, np.full((Hn, Wn), 0.01), np.full((Hn, Wn), b), np.full((Hn, Wn), 1e-4),
         np.full((Hn, Wn), c), np.full((Hn, Wn), 4e-4)]
    fx = 512.0
    mu, vmu, gx, vgx, gy, vgy = network_priors(m, W, H, fx=fx, focal_ref=fx * Wn / W)   # no shift
    un = (np.arange(W) + 0.5) * Wn / W - 0.5
    vn = (np.arange(H) + 0.5) * Hn / H - 0.5
    inner = (slice(4, H - 4), slice(4, W - 4))
    assert np.allclose(mu[inner], (a + b * un[None, :] + c * vn[:, None])[inner], atol=1e-13)
    fdx = mu[:, 1:] - mu[:, :-1]
    fdy = mu[1:, :] - mu[:-1, :]
    assert np.allclose(fdx[4:-4, 4:-4], gx[4:-4, 4:-5], atol=1e-13)
    assert np.allclose(fdy[4:-4, 4:-4], gy[4:-5, 4:-4], atol=1e-13)
    assert np.allclose(vgx, 1e-4 * (Wn / W) ** 2) and np.allclose(vgy, 4e-4 * (Hn / H) ** 2)
    assert np.allclose(vmu, 0.01)


def test_focal_length_shifts_the_log_depth_only():
    m = _maps(24, 32, seed=3)
    a = network_priors(m, 40, 30, fx=200.0, focal_ref=100.0)
    b = network_priors(m, 40, 30, fx=400.0, focal_ref=100.0)
    assert np.allclose(b[0] - a[0], np.log(2.0), atol=1e-14)
    for k in range(1, 6):
        assert np.array_equal(a[k], b[k])
    # the shift is the log of the focal length at the network's size over the reference
    c = network_priors(m, 32, 24, fx=150.0, focal_ref=150.0)
    assert np.allclose(c[0], m[0])
