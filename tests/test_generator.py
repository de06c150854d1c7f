"""Seeded generator: determinism, ranges, prior statistics."""

import numpy as np

import kfsynth


def test_same_seed_same_bytes():
    a = kfsynth.make_case(12345, 64, 48, 2, "walk")
    b = kfsynth.make_case(12345, 64, 48, 2, "walk")
    assert np.array_equal(a.image0, b.image0)
    for x, y in zip(a.images, b.images):
        assert np.array_equal(x, y)
    for x, y in zip(a.priors.maps(), b.priors.maps()):
        assert np.array_equal(x, y)
    for x, y in zip(a.poses, b.poses):
        assert np.array_equal(x, y)
    c = kfsynth.make_case(12346, 64, 48, 2, "walk")
    assert not np.array_equal(a.image0, c.image0)


def test_ranges_and_camera(case_c0):
    c = case_c0
    assert c.image0.dtype == np.uint8 and c.image0.shape == (120, 160)
    assert c.depth0.min() >= 0.5 and c.depth0.max() <= 5.0
    assert np.allclose(c.K, [[128, 0, 80], [0, 128, 60], [0, 0, 1]])
    assert len(c.poses) == 1 and len(c.images) == 1
    T = c.poses[0]
    assert abs(np.linalg.norm(T[:3, 3]) - 0.05) < 1e-12
    R = T[:3, :3]
    ang = np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    assert abs(ang - 1.0) < 1e-9
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)


def test_prior_statistics():
    c = kfsynth.make_case(777, 160, 120, 1)
    p = c.priors
    x = np.log(c.depth0)
    z = (p.logdepth - x) / np.sqrt(p.logdepth_var)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.03
    s = np.sqrt(p.logdepth_var)
    assert s.min() >= 0.02 - 1e-12 and s.max() <= 0.3 + 1e-12
    gx_true = x[:, 1:] - x[:, :-1]
    zg = (p.gx[:, :-1] - gx_true) / np.sqrt(p.gx_var[:, :-1])
    assert abs(zg.mean()) < 0.03 and abs(zg.std() - 1) < 0.03
    sg = np.sqrt(p.gy_var)
    assert sg.min() >= 0.01 - 1e-12 and sg.max() <= 0.2 + 1e-12


def test_walk_steps():
    c = kfsynth.make_case(4321, 64, 48, 5, "walk")
    prev = np.eye(4)
    for T in c.poses:
        assert abs(np.linalg.norm(T[:3, 3] - prev[:3, 3]) - 0.02) < 1e-12
        dR = prev[:3, :3].T @ T[:3, :3]
        ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
        assert abs(ang - 0.5) < 1e-6
        prev = T


def test_translation_scale_only_scales_translation():
    a = kfsynth.make_case(99, 64, 48, 1, translation_scale=1.0)
    b = kfsynth.make_case(99, 64, 48, 1, translation_scale=2.0)
    assert np.array_equal(a.images[0], b.images[0])
    assert np.allclose(b.poses[0][:3, 3] * 2.0, a.poses[0][:3, 3], rtol=0, atol=0)
