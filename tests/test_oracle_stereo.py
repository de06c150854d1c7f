"""Pins of the semi-dense oracle (Sec. II-B) against geometry, closed forms and statistics."""

import math

import numpy as np
import pytest

import kfsynth
from oracle import geometry, stereo
from oracle.stereo import StereoParams, UPDATED


def _random_pose(rng, t_scale=0.05, r_deg=2.0):
    a = rng.standard_normal(3)
    u = rng.standard_normal(3)
    R = kfsynth.so3_exp(math.radians(r_deg) * a / np.linalg.norm(a))
    return kfsynth.pose_matrix(R, t_scale * u / np.linalg.norm(u))


def test_projection_matches_backproject_transform_project():
    """pi(H x~ + rho b) equals back-projection, T_WC1^-1 T_WC0, projection (Sec. II-B eq.)."""
    rng = np.random.default_rng(3)
    K = kfsynth.camera_matrix(320, 240)
    for _ in range(20):
        T0 = _random_pose(rng, 0.3, 10)
        T1 = _random_pose(rng, 0.3, 10)
        Hinf, b, _ = geometry.epipolar_constants(K, T0, T1)
        u, v = rng.uniform(0, 319), rng.uniform(0, 239)
        d = rng.uniform(0.5, 5)
        px, py, X2 = geometry.project_through(Hinf, b, u, v, 1.0 / d)
        qx, qy = geometry.project_point(K, T0, T1, u, v, d)
        assert X2 > 0
        assert abs(px - qx) < 1e-9 and abs(py - qy) < 1e-9


def test_keyframe_epipole_is_image_of_new_camera_centre():
    rng = np.random.default_rng(5)
    K = kfsynth.camera_matrix(160, 120)
    for _ in range(10):
        T1 = _random_pose(rng)
        T0 = np.eye(4)
        _, _, e0 = geometry.epipolar_constants(K, T0, T1)
        c1 = T1[:3, 3]                       # camera-1 centre in world = keyframe frame
        e_ref = K @ c1
        assert np.allclose(e0 / np.linalg.norm(e0), e_ref / np.linalg.norm(e_ref), atol=1e-12)


def _stereo_pair(ramp=False, D=6, W=64, H=16, seed=0):
    """Pure x-translation by B = 0.25 m, R = I, fx = 32: disparity = 8 rho (P8/P9 setups).

    With d_near = 0.5 and d_far = 8 the segment spans disparities 1..16, so 16
    samples fall on integer disparities k + 1.
    """
    rng = np.random.default_rng(seed)
    K = np.array([[32.0, 0, 32.0], [0, 32.0, 8.0], [0, 0, 1.0]])
    T0 = np.eye(4)
    T1 = kfsynth.pose_matrix(np.eye(3), np.array([0.25, 0.0, 0.0]))
    if ramp:
        uu = np.tile(np.arange(W), (H, 1))
        I0 = (8 * uu).clip(0, 255).astype(np.uint8)
        I1 = (8 * uu + 52).clip(0, 255).astype(np.uint8)     # I1(u') = I0(u' + 6.5)
    else:
        I0 = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
        I1 = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
        I1[:, : W - D] = I0[:, D:]                            # I1(u') = I0(u' + D)
    return K, T0, T1, I0, I1


@pytest.mark.parametrize("pattern", ["line5", "sq5x5"])
def test_integer_disparity_exact_match(pattern):
    """P8: fronto-parallel shift by D px -> k* = D - 1, SSD 0, lambda* = 0, d* = 8 / D."""
    D = 6
    K, T0, T1, I0, I1 = _stereo_pair(D=D)
    H, W = I0.shape
    sp = StereoParams(n_samples=16, pattern=pattern, d_near=0.5, d_far=8.0)
    mask = stereo.texture_mask(I0, sp.grad_gate)
    z = np.zeros((H, W))
    res = stereo.epipolar_search(I0, I1, K, T0, T1, z, z, np.zeros((H, W), bool), mask, sp)
    u = res.pix % W
    sel = (u >= D + 2) & (u <= W - 3)
    assert sel.sum() > 100
    assert np.all(res.status[sel] == UPDATED)
    assert np.all(res.k_best[sel] == D - 1)
    rows = np.flatnonzero(sel)
    assert np.all(res.ssd[rows, D - 1] == 0.0)
    assert np.all(res.lam[sel] == 0.0)
    assert np.all(res.d_star[sel] == 1.0 / (D / 8.0))
    # every other valid sample has a positive SSD (random texture)
    other = np.delete(res.ssd[rows], D - 1, axis=1)
    assert np.all(other > 0)


@pytest.mark.parametrize("pattern,P", [("line5", 5), ("sq5x5", 25)])
def test_ramp_variance_closed_form(pattern, P):
    """P9: linear ramp of slope 8 along the epipolar line: de = 8 h 1, sigma_d^2 = dd^2/(P 64 h^2).

    The true disparity 6.5 lies halfway between samples k = 5 (D = 6) and k = 6 (D = 7):
    SSD ties -> k* = 5 (smallest), n* = 6, lambda* = 1/2 exactly.
    """
    K, T0, T1, I0, I1 = _stereo_pair(ramp=True, W=32)
    H, W = I0.shape
    sp = StereoParams(n_samples=16, pattern=pattern, d_near=0.5, d_far=8.0)
    mask = stereo.texture_mask(I0, sp.grad_gate)
    z = np.zeros((H, W))
    res = stereo.epipolar_search(I0, I1, K, T0, T1, z, z, np.zeros((H, W), bool), mask, sp)
    u = res.pix % W
    sel = (u >= 10) & (u <= 28)
    assert sel.sum() > 20
    assert np.all(res.status[sel] == UPDATED)
    assert np.all(res.k_best[sel] == 5) and np.all(res.k_nbr[sel] == 6)
    assert np.all(res.lam[sel] == 0.5)
    d_a, d_b = 8.0 / 6.0, 8.0 / 7.0
    assert np.allclose(res.d_star[sel], d_a + 0.5 * (d_b - d_a), rtol=1e-15, atol=0)
    expect = (d_b - d_a) ** 2 / (P * 64.0 * 1.0)
    assert np.allclose(res.var_d[sel], expect, rtol=1e-13, atol=0)


def test_translation_scale_metamorphic():
    """P7 (stereo side): translation / 2 and depth range / 2 -> same matches, d* / 2, var / 4."""
    c = kfsynth.config_case(0, 0)
    sp = StereoParams(n_samples=32, pattern="line5")
    sp2 = StereoParams(n_samples=32, pattern="line5", d_near=sp.d_near / 2, d_far=sp.d_far / 2)
    T1 = c.poses[0]
    T1h = T1.copy()
    T1h[:3, 3] /= 2.0
    mask = stereo.texture_mask(c.image0)
    z = np.zeros((c.H, c.W))
    f = np.zeros((c.H, c.W), bool)
    a = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, T1, z, z, f, mask, sp)
    b = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, T1h, z, z, f, mask, sp2)
    assert np.array_equal(a.status, b.status)
    ok = a.status == UPDATED
    assert np.array_equal(a.k_best[ok], b.k_best[ok])
    assert np.allclose(b.d_star[ok], a.d_star[ok] / 2, rtol=1e-12)
    assert np.allclose(b.var_d[ok], a.var_d[ok] / 4, rtol=1e-11)


def test_brute_force_argmin_and_neighbour_rule():
    """k* is the first minimum of all N_s SSDs; n* the lower valid neighbour, ties to k*-1."""
    c = kfsynth.config_case(0, 0)
    sp = StereoParams(n_samples=32, pattern="line5")
    mask = stereo.texture_mask(c.image0)
    z = np.zeros((c.H, c.W))
    res = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], z, z,
                                 np.zeros((c.H, c.W), bool), mask, sp)
    ok = np.flatnonzero(res.status == UPDATED)
    for r in ok[:: max(1, ok.size // 400)]:
        s = res.ssd[r]
        k = int(np.flatnonzero(s == s.min())[0])
        assert res.k_best[r] == k
        left = s[k - 1] if k > 0 else np.inf
        right = s[k + 1] if k < sp.n_samples - 1 else np.inf
        assert res.k_nbr[r] == (k - 1 if left <= right else k + 1)
        assert 0.0 <= res.lam[r] <= 1.0


def test_depth_accuracy_on_rendered_scene(case_c0):
    """Geometry sanity on a rendered scene: most matches land near the true depth."""
    c = case_c0
    sp = StereoParams(n_samples=32, pattern="line5")
    mask = stereo.texture_mask(c.image0)
    z = np.zeros((c.H, c.W))
    res = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], z, z,
                                 np.zeros((c.H, c.W), bool), mask, sp)
    ok = res.status == UPDATED
    assert ok.mean() > 0.9
    gt = c.depth0.ravel()[res.pix[ok]]
    rel = np.abs(res.d_star[ok] - gt) / gt
    assert np.median(rel) < 0.08
    assert np.mean(rel < 0.1) > 0.8


def test_interval_search_after_first_observation(case_c0):
    """A valid filter state centres the sample grid on rho (interval rho +- 2 sigma, Sec. II-B).

    With N_s samples at 1-px steps the grid spans more than a narrow interval
    (reading R5), so the check is on the centring: samples k = N_s/2 - 1 and
    N_s/2 straddle the image of the interval centre.
    """
    c = case_c0
    sp = StereoParams(n_samples=32, pattern="line5")
    mask = stereo.texture_mask(c.image0)
    H, W = c.H, c.W
    rho_true = 1.0 / c.depth0
    var = np.full((H, W), (0.02 * rho_true) ** 2)
    res = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], rho_true, var,
                                 np.ones((H, W), bool), mask, sp)
    ok = res.status == UPDATED
    assert ok.mean() > 0.9
    rt = rho_true.ravel()[res.pix[ok]]
    mid = 0.5 * (res.rho_k[ok, 15] + res.rho_k[ok, 16])
    assert np.max(np.abs(mid / rt - 1)) < 0.01
    rk = res.rho_k[ok]
    fin = np.isfinite(res.ssd[ok])
    assert np.all(rk[fin] >= 1 / sp.d_far) and np.all(rk[fin] <= 1 / sp.d_near)
    gt = c.depth0.ravel()[res.pix[ok]]
    rel = np.abs(res.d_star[ok] - gt) / gt
    assert np.median(rel) < 0.08


def test_converged_filter_stops_searching():
    """A variance so small that the interval's image is under 1e-6 px skips the pixel."""
    c = kfsynth.make_case(31, 64, 48, 1)
    sp = StereoParams(n_samples=16, pattern="sq5x5")
    mask = stereo.texture_mask(c.image0)
    rho = 1.0 / c.depth0
    res = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], rho,
                                 np.full(rho.shape, 1e-24), np.ones(rho.shape, bool), mask, sp)
    assert np.all(res.status == stereo.DEGENERATE_LINE)


def test_filter_gaussian_product_algebra():
    """P10: information form; n identical observations divide the variance by n."""
    rng = np.random.default_rng(0)
    H, W = 4, 5
    rho = rng.uniform(0.2, 2, (H, W))
    var = rng.uniform(1e-4, 1e-2, (H, W))
    valid = rng.random((H, W)) < 0.5
    pix = np.arange(H * W)
    ro = rng.uniform(0.2, 2, H * W)
    vo = rng.uniform(1e-4, 1e-2, H * W)
    r2, v2, ok2 = stereo.filter_update(rho, var, valid, pix, ro, vo)
    info = np.where(valid.ravel(), 1 / var.ravel(), 0) + 1 / vo
    mean = (np.where(valid.ravel(), rho.ravel() / var.ravel(), 0) + ro / vo) / info
    assert np.allclose(v2.ravel(), 1 / info, rtol=1e-13)
    assert np.allclose(r2.ravel(), mean, rtol=1e-13)
    assert ok2.all()
    # repeated identical observation
    r, v, ok = np.zeros((1, 1)), np.zeros((1, 1)), np.zeros((1, 1), bool)
    for n in range(1, 9):
        r, v, ok = stereo.filter_update(r, v, ok, np.array([0]), np.array([0.7]), np.array([0.04]))
        assert abs(v[0, 0] - 0.04 / n) < 1e-15 and abs(r[0, 0] - 0.7) < 1e-15


def test_log_conversion_delta_method():
    """P11: z = -ln rho and R = v / rho^2 agree with the spread of -ln(rho + noise)."""
    rng = np.random.default_rng(1)
    rho0, sd = 0.8, 0.004
    samp = -np.log(rho0 + sd * rng.standard_normal(1_000_000))
    z, R, ok = stereo.log_measurements(np.array([[rho0]]), np.array([[sd * sd]]), np.array([[True]]))
    assert abs(z[0, 0] - (-math.log(rho0))) < 1e-15
    assert abs(samp.var() / R[0, 0] - 1) < 0.01
    assert abs(samp.mean() - z[0, 0]) < 1e-4
    _, Rf, _ = stereo.log_measurements(np.array([[1.0]]), np.array([[1e-12]]), np.array([[True]]), r_floor=1e-6)
    assert Rf[0, 0] == 1e-6


def test_float32_decisions_agree_with_float64_outside_ties(case_c0):
    """The float32 mode changes only near-tie argmins (reading: decisions in kernel precision)."""
    c = case_c0
    sp = StereoParams(n_samples=32, pattern="line5")
    mask = stereo.texture_mask(c.image0)
    z = np.zeros((c.H, c.W))
    f = np.zeros((c.H, c.W), bool)
    a = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], z, z, f, mask, sp)
    b = stereo.epipolar_search(c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], z, z, f, mask, sp,
                               dtype=np.float32)
    ok = (a.status == UPDATED) & (b.status == UPDATED)
    s = np.sort(a.ssd[ok], axis=1)
    margin = s[:, 1] - s[:, 0]
    clear = margin >= 1e-3 * (1 + s[:, 0]) + 0.05 * 5
    assert clear.mean() > 0.95
    assert np.array_equal(a.k_best[ok][clear], b.k_best[ok][clear])
    assert np.mean(a.status == b.status) > 0.999


# ------------------------------------------------------------------ pins of the texture gate,
# the bilinear sampler at fractional positions and the direction of the sub-pixel step

def _gate_image(a, b, H=16, W=20):
    """uint8 image whose central differences are exactly I[u+1]-I[u-1] = a and I[v+1]-I[v-1] = b
    everywhere inside: I = floor(a u / 2) + floor(b v / 2) (steps alternate for odd a, b)."""
    uu, vv = np.meshgrid(np.arange(W), np.arange(H))
    return (np.floor(a * uu / 2.0) + np.floor(b * vv / 2.0)).astype(np.uint8)


def test_texture_gate_threshold_is_on_the_halved_gradient_norm():
    """R1 (Sec. II-B, 'sufficient texture'): |((I[u+1]-I[u-1])/2, (I[v+1]-I[v-1])/2)| >= 6.

    Cases and the mistakes each one catches:
    - ramp I = 6u: halved difference exactly 6 -> textured (a strict '>' gate fails);
    - ramp with steps 5, 6, 5, ...: halved difference 5.5 -> not textured (a gate on the
      un-halved difference 11 fails, and so does a gate on |grad|^2 >= 6, since 5.5^2 >= 6);
    - a = 8, b = 9: (4, 4.5), norm sqrt(36.25) -> textured (a max-norm or x-only gate fails);
    - a = 7, b = 9: (3.5, 4.5), norm sqrt(32.5) -> not textured (an L1 gate, 8 >= 6, fails).
    """
    inner = (slice(2, -2), slice(2, -2))
    for a, b, textured in ((12, 0, True), (11, 0, False), (8, 9, True), (7, 9, False), (0, 12, True),
                           (0, 11, False)):
        I = _gate_image(a, b)
        m = stereo.texture_mask(I, 6.0, 2)
        assert np.all(m[inner] == textured), (a, b)
    # exactly on the gate in x alone: I = 6u has I[u+1] - I[u-1] = 12
    assert np.array_equal(_gate_image(12, 0), (6 * np.tile(np.arange(20), (16, 1))).astype(np.uint8))


def test_texture_gate_border_is_two_pixels():
    """R1: a border of 2 px is never searched; the third row / column is (a border of 1 or 3 fails)."""
    I = _gate_image(20, 20, H=12, W=14)
    m = stereo.texture_mask(I, 6.0, 2)
    H, W = I.shape
    expect = np.zeros((H, W), bool)
    expect[2:H - 2, 2:W - 2] = True
    assert np.array_equal(m, expect)


def test_bilinear_reproduces_bilinear_functions_at_fractional_points():
    """Bilinear interpolation is exact on I(u, v) = a + b u + c v + d u v, at any fractional point,
    including points in the last cell (u in [W-2, W-1], v in [H-2, H-1]) and on its far edges,
    where the cell origin is clamped to W-2 / H-2. Swapping the u and v fractions (f <-> g), the
    weights of I10 and I01, or dropping the clamp all fail."""
    rng = np.random.default_rng(11)
    H, W = 9, 13
    uu, vv = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    for _ in range(5):
        a, b, c, d = rng.uniform(-3, 3, 4)
        img = a + b * uu + c * vv + d * uu * vv
        u = np.concatenate([rng.uniform(0, W - 1, 400), rng.uniform(W - 2, W - 1, 50), [W - 1.0, 0.0, W - 1.0]])
        v = np.concatenate([rng.uniform(0, H - 1, 400), rng.uniform(H - 2, H - 1, 50), [H - 1.0, H - 1.0, 0.0]])
        got = stereo.bilinear(img, u, v)
        assert np.allclose(got, a + b * u + c * v + d * u * v, rtol=0, atol=1e-12)
    # an image that is linear in u only must not depend on the v fraction (catches f <-> g)
    img = np.tile(np.arange(W, dtype=np.float64) * 5.0, (H, 1))
    assert np.allclose(stereo.bilinear(img, np.array([3.25]), np.array([4.75])), [16.25], atol=1e-13)


@pytest.mark.parametrize("pattern,P", [("line5", 5), ("sq5x5", 25)])
def test_subpixel_step_direction_on_an_asymmetric_ramp(pattern, P):
    """R6 (Sec. II-B, interpolation between two steps), asymmetric case.

    I1(u') = I0(u' + 6.25) on a ramp of slope 8: sample k sits at disparity k + 1, so every
    pattern point has e_k = 8 (6.25 - (k + 1)) = 42 - 8 k: e_5 = 2, e_6 = -6, e_4 = 10.
    Then k* = 5, n* = 6 (SSD 36 P < 100 P), de = -8, lambda* = -(2)(-8) / 64 = 1/4 exactly,
    d* = d_a + (d_b - d_a) / 4 with d_a = 8/6, d_b = 8/7 (linear in depth), and
    sigma_d^2 = (d_b - d_a)^2 / (64 P).
    Mistakes caught: interpolating from n* towards k* (lambda 3/4 from d_b), the opposite sign of
    lambda (clipped to 0), interpolating in inverse depth, taking the higher-SSD neighbour.
    """
    K, T0, T1, I0, _ = _stereo_pair(ramp=True, W=32)
    H, W = I0.shape
    uu = np.tile(np.arange(W), (H, 1))
    I1 = (8 * uu + 50).clip(0, 255).astype(np.uint8)            # I1(u') = I0(u' + 6.25)
    sp = StereoParams(n_samples=16, pattern=pattern, d_near=0.5, d_far=8.0)
    mask = stereo.texture_mask(I0, sp.grad_gate)
    z = np.zeros((H, W))
    res = stereo.epipolar_search(I0, I1, K, T0, T1, z, z, np.zeros((H, W), bool), mask, sp)
    u = res.pix % W
    sel = (u >= 10) & (u <= 28)
    assert sel.sum() > 20
    assert np.all(res.status[sel] == UPDATED)
    rows = np.flatnonzero(sel)
    assert np.all(res.ssd[rows, 5] == 4.0 * P) and np.all(res.ssd[rows, 6] == 36.0 * P)
    assert np.all(res.ssd[rows, 4] == 100.0 * P)
    assert np.all(res.k_best[sel] == 5) and np.all(res.k_nbr[sel] == 6)
    assert np.all(res.lam[sel] == 0.25)
    d_a, d_b = 8.0 / 6.0, 8.0 / 7.0
    assert np.allclose(res.d_star[sel], d_a + 0.25 * (d_b - d_a), rtol=1e-15, atol=0)
    assert np.allclose(res.var_d[sel], (d_b - d_a) ** 2 / (64.0 * P), rtol=1e-13, atol=0)


def test_search_in_row_blocks_equals_one_call(case_c0):
    """Searching the texture mask in row blocks (another executor, as the GPU
    comparisons do with a process pool) concatenates to exactly the one-call
    result, first frame and with a filter state; each block's pixels are searched
    by the same function on the whole images."""
    import concurrent.futures
    from oracle.pipeline import search_in_blocks
    c = case_c0
    sp = StereoParams(n_samples=32, pattern="sq5x5")
    mask = stereo.texture_mask(c.image0)
    z = np.zeros((c.H, c.W))
    args = (c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], z, z, np.zeros((c.H, c.W), bool), mask, sp)
    one = stereo.epipolar_search(*args)
    with concurrent.futures.ThreadPoolExecutor(3) as ex:
        blk = search_in_blocks(ex, 5, *args)
        r, v, ok = stereo.filter_update(z, z, np.zeros((c.H, c.W), bool), one.pix[one.status == UPDATED],
                                        one.rho_obs[one.status == UPDATED], one.var_obs[one.status == UPDATED])
        args2 = (c.image0, c.images[0], c.K, c.T_wc0, c.poses[0], r, v, ok, mask, sp)
        one2 = stereo.epipolar_search(*args2)
        blk2 = search_in_blocks(ex, 7, *args2)
    for a, b in ((one, blk), (one2, blk2)):
        for f in stereo.SearchResult.__dataclass_fields__:
            assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_keyframe_decision_rule():
    """Sec. II keyframe rule: translation beyond lambda_trans or inliers below
    lambda_inliers ask for a new keyframe; strict comparisons; 0 disables a test.
    The translation is the distance between camera centres, whatever the
    rotations (a rotation about the keyframe centre moves nothing)."""
    from oracle.pipeline import NEW_KF_INLIERS, NEW_KF_TRANSLATION, camera_translation, keyframe_decision
    R = kfsynth.so3_exp(np.array([0.3, -0.2, 0.5]))
    T0 = kfsynth.pose_matrix(R, np.array([1.0, 2.0, 3.0]))
    T1 = kfsynth.pose_matrix(R.T, np.array([1.0, 2.0, 3.0]) + np.array([0.03, -0.04, 0.0]))
    assert abs(camera_translation(T0, T1) - 0.05) < 1e-15
    assert camera_translation(T0, kfsynth.pose_matrix(np.eye(3), T0[:3, 3])) == 0.0
    assert keyframe_decision(0.05, 100, 0.05, 100) == 0
    assert keyframe_decision(0.0500001, 100, 0.05, 100) == NEW_KF_TRANSLATION
    assert keyframe_decision(0.05, 99, 0.05, 100) == NEW_KF_INLIERS
    assert keyframe_decision(1.0, 0, 0.5, 1) == NEW_KF_TRANSLATION | NEW_KF_INLIERS
    assert keyframe_decision(1e9, 0, 0.0, 0) == 0


def test_oracle_keyframe_skips_fusion_on_a_new_keyframe(case_c0):
    """When the rule fires, the semi-dense filter is updated but the depth map
    keeps its last fused state."""
    from oracle import OracleKeyframe, SolverParams
    from oracle.pipeline import NEW_KF_INLIERS
    c = case_c0
    ok = OracleKeyframe(c.K, c.W, c.H, StereoParams(n_samples=32, pattern="line5"),
                        SolverParams(n_gn=2, linear_solver="direct"), lambda_inliers=10 ** 9)
    ok.set_prior(c.image0, *c.priors.maps(), c.T_wc0)
    rep = ok.fuse_frame(c.images[0], c.poses[0])
    assert rep.new_keyframe == NEW_KF_INLIERS and rep.n_updated > 0 and ok.valid.sum() == rep.n_updated
    assert np.array_equal(ok.x, c.priors.logdepth) and ok.tau == 0.0
