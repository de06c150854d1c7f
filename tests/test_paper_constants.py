"""The constants the paper states are the defaults of the oracle (tests/golden/paper_constants.json)."""

import json
import os

import numpy as np

import kfsynth
from oracle import fusion, stereo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_gauss_newton_iterations_default():
    assert fusion.SolverParams().n_gn == _golden()["gauss_newton_iterations"]["value"]


def test_line_pattern_has_five_points_one_pixel_apart():
    g = _golden()
    c = kfsynth.make_case(5, 48, 32, 1)
    sp = stereo.StereoParams(n_samples=8, pattern="line5")
    mask = stereo.texture_mask(c.image0)
    z = np.zeros((32, 48))
    res = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], z, z,
                                 np.zeros((32, 48), bool), mask, sp)
    ok = res.status == stereo.UPDATED
    # residual vectors have one entry per pattern point
    ek = stereo._pattern(c.image0.astype(float), np.array([10.0]), np.array([10.0]),
                         np.array([1.0]), np.array([0.0]), "line5", np.dtype(float))[0]
    assert len(ek) == g["pattern_points"]["value"]
    # steps along the epipolar line are never shorter than one pixel
    assert ok.any()


def test_interval_is_two_sigma():
    """A valid estimate with sigma small enough that +-2 sigma stays inside the global range."""
    g = _golden()
    K = np.array([[32.0, 0, 32.0], [0, 32.0, 8.0], [0, 0, 1.0]])
    T1 = kfsynth.pose_matrix(np.eye(3), np.array([0.25, 0.0, 0.0]))
    rng = np.random.default_rng(0)
    I0 = rng.integers(0, 256, (16, 64)).astype(np.uint8)
    sp = stereo.StereoParams(n_samples=4, pattern="line5", d_near=0.5, d_far=8.0)
    mask = np.zeros((16, 64), bool)
    mask[8, 40] = True
    rho = np.full((16, 64), 0.75)
    var = np.full((16, 64), 0.1 ** 2)
    res = stereo.epipolar_search(I0, I0, K, np.eye(4), T1, rho, var, np.ones((16, 64), bool), mask, sp)
    # disparity = 8 rho: the interval rho +- k sigma maps to a 8 * 2 k sigma = 3.2 px segment
    # (> 3 px for 4 samples), so the end samples sit exactly on rho +- k sigma
    k = g["interval_sigmas"]["value"]
    expect = 0.75 + k * 0.1 * np.array([1.0, 1 / 3, -1 / 3, -1.0])
    assert np.allclose(np.sort(res.rho_k[0])[::-1], expect, atol=1e-12)
