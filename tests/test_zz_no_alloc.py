"""kf_fuse_frame_static (no allocation: scratch in a fixed device array) against
kf_fuse_frame, through the C ABI, on two calls in a row -- the second on a
smaller keyframe, so it runs on what the first call left in the array."""

import ctypes

import numpy as np
import pytest

import kfsynth

import gpu_util as gu

pytestmark = pytest.mark.gpu


def _pair(case, precision, pattern, ns):
    a = gu.make_gpu_kf(case, precision, pattern, ns)
    b = gu.make_gpu_kf(case, precision, pattern, ns)
    return a, b


@pytest.mark.parametrize("precision,pattern,ns", [("f32", "sq5x5", 64), ("f64", "line5", 32)])
def test_fuse_frame_static_equals_fuse_frame(precision, pattern, ns):
    from paper_2207_12244_amd import kf as K
    t = gu.torch()
    lib = K.load_library()
    cases = [kfsynth.config_case(1, 0, frames=2), kfsynth.config_case(0, 0, frames=2)]   # 320x240, then 160x120
    for case in cases:
        gu.say(f"[no-alloc] {case.W}x{case.H} {precision} {pattern} N_s={ns}")
        ref, sta = _pair(case, precision, pattern, ns)
        for f in range(2):
            img = gu.dev(case.images[f], t.uint8)
            ref.fuse_frame(img, case.poses[f])
            st = lib.kf_fuse_frame_static(sta.ctx, ctypes.c_void_p(img.data_ptr()), K._pose(case.poses[f]))
            assert st == K.KF_OK, lib.kf_last_error(sta.ctx)
        a, b = gu.np_state(ref), gu.np_state(sta)
        for k in ("x", "rho", "var", "match"):
            assert np.array_equal(a[k], b[k]), k
        assert a["tau"] == b["tau"]
        assert ref.stats().team_syncs == sta.stats().team_syncs
        ref.close()
        sta.close()


def test_fuse_frame_static_rejects_oversized_keyframes():
    """A valid keyframe whose scratch exceeds the static array: 8000 x 96 with an
    explicit 8 x 32 tiling at 1024 threads (tiles of 1000 x 3 px, so 256 tile
    boundaries of 2 x 2006 slots: ~33 MB of exchange words) is refused before
    any device work, and the context stays usable."""
    from paper_2207_12244_amd import kf as K
    from paper_2207_12244_amd.kf import Keyframe
    t = gu.torch()
    lib = K.load_library()
    W, H = 8000, 96
    kf = Keyframe(W, H, precision="f32", pattern="line5", n_samples=32, tiles=(8, 32), solver_threads=1024)
    z = t.zeros((H, W), dtype=t.float32, device="cuda")
    kf.set_prior(t.zeros((H, W), dtype=t.uint8, device="cuda"), z, z + 1, z, z + 1, z, z + 1, np.eye(4))
    img = t.zeros((H, W), dtype=t.uint8, device="cuda")
    st = lib.kf_fuse_frame_static(kf.ctx, ctypes.c_void_p(img.data_ptr()), K._pose(np.eye(4)))
    assert st == K.KF_ERR_ARG and b"static array" in lib.kf_last_error(kf.ctx)
    kf.read_depth()
    kf.close()
