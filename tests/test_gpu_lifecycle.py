"""Keyframe rule (Sec. II) on the GPU against the oracle keyframe: a frame whose
camera centre moved more than lambda_trans from the keyframe's, or whose
semi-dense update produced fewer than lambda_inliers measurements, updates the
filter but is not fused. Decisions are compared frame by frame over a walk, the
depth map must stay bit-identical on frames that ask for a new keyframe, and a
new prior (kf_set_prior) starts the next keyframe."""

import numpy as np
import pytest

import kfsynth
from oracle import OracleKeyframe, SolverParams, StereoParams
from oracle.pipeline import NEW_KF_INLIERS, NEW_KF_TRANSLATION, camera_translation

import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_translation_rule_over_a_walk():
    case = kfsynth.config_case(1, 0, frames=10)
    dist = [camera_translation(case.T_wc0, T) for T in case.poses]
    # a threshold half way between two frames' distances, so both sides decide alike
    srt = sorted(dist)
    lam = 0.5 * (srt[4] + srt[5])
    gu.say(f"[lifecycle] 320x240 f32 walk, distances {np.round(dist, 4).tolist()}, lambda_trans {lam:.4f}")
    from paper_2207_12244_amd.kf import Keyframe
    t = gu.torch()
    kf = Keyframe(case.W, case.H, precision="f32", pattern="sq5x5", n_samples=64, n_gn=10, n_cg=20, K=case.K,
                  lambda_trans=lam)
    kf.set_prior(gu.dev(case.image0, t.uint8), *[gu.dev(m, t.float32) for m in case.priors.maps()], case.T_wc0)
    ok = OracleKeyframe(case.K, case.W, case.H, StereoParams(n_samples=64, pattern="sq5x5"),
                        SolverParams(n_gn=10, n_cg=20, linear_solver="pcg"), lambda_trans=lam)
    ok.set_prior(case.image0, *case.priors.maps(), case.T_wc0)
    fired = 0
    for f in range(len(case.images)):
        before = gu.np_state(kf)
        kf.fuse_frame(gu.dev(case.images[f], t.uint8), case.poses[f])
        st = gu.np_state(kf)
        s = kf.stats()
        rep = ok.fuse_frame(case.images[f], case.poses[f])
        gu.say(f"[lifecycle] frame {f + 1}: distance {dist[f]:.4f} gpu {s.new_keyframe} oracle {rep.new_keyframe} "
               f"syncs {s.team_syncs}")
        assert s.new_keyframe == rep.new_keyframe
        if rep.new_keyframe:
            fired += 1
            assert rep.new_keyframe == NEW_KF_TRANSLATION
            assert np.array_equal(st["x"], before["x"]) and st["tau"] == before["tau"]
            assert s.team_syncs == 0
            assert np.count_nonzero(st["var"] != before["var"]) > 0      # the filter was still updated
        else:
            assert s.team_syncs > 0
    assert 0 < fired < len(case.images)
    # the caller starts the next keyframe: the rule measures from the new keyframe's pose
    kf.set_prior(gu.dev(case.images[0], t.uint8), *[gu.dev(m, t.float32) for m in case.priors.maps()],
                 case.poses[0])
    kf.fuse_frame(gu.dev(case.images[1], t.uint8), case.poses[1])
    assert kf.stats().new_keyframe == (NEW_KF_TRANSLATION if camera_translation(case.poses[0], case.poses[1]) > lam
                                       else 0)
    kf.close()


@pytest.mark.parametrize("lam,expect", [(1, 0), (10 ** 9, NEW_KF_INLIERS)])
def test_inlier_rule(lam, expect):
    case = kfsynth.config_case(0, 0)
    gu.say(f"[lifecycle] 160x120 f64 lambda_inliers {lam}")
    from paper_2207_12244_amd.kf import Keyframe
    t = gu.torch()
    kf = Keyframe(case.W, case.H, precision="f64", pattern="line5", n_samples=32, n_gn=3, n_cg=15, K=case.K,
                  lambda_inliers=lam)
    kf.set_prior(gu.dev(case.image0, t.uint8), *[gu.dev(m, t.float64) for m in case.priors.maps()], case.T_wc0)
    kf.fuse_frame(gu.dev(case.images[0], t.uint8), case.poses[0])
    st = gu.np_state(kf)
    s = kf.stats()
    assert s.new_keyframe == expect and s.n_updated > 0
    if expect:
        assert np.array_equal(st["x"], case.priors.logdepth) and st["tau"] == 0.0
    else:
        assert not np.array_equal(st["x"], case.priors.logdepth)
    kf.close()


def test_rule_per_member_in_a_batch():
    """Batched members decide on their own: one member with an unreachable inlier
    threshold is left unfused, the others fuse as they would alone."""
    from paper_2207_12244_amd.kf import Batch, Keyframe
    t = gu.torch()
    cases = [kfsynth.config_case(3, i, size_index=i % 2) for i in range(3)]
    members, imgs, poses = [], [], []
    for i, c in enumerate(cases):
        kf = Keyframe(c.W, c.H, precision="f32", pattern="line5", n_samples=32, n_gn=10, n_cg=20, K=c.K,
                      solver_threads=512, lambda_inliers=10 ** 9 if i == 1 else 0)
        kf.set_prior(gu.dev(c.image0, t.uint8), *[gu.dev(m, t.float32) for m in c.priors.maps()], c.T_wc0)
        members.append(kf)
        imgs.append(gu.dev(c.images[0], t.uint8))
        poses.append(c.poses[0])
    batch = Batch(members)
    batch.fuse(imgs, poses)
    for i, (kf, c) in enumerate(zip(members, cases)):
        s = kf.stats()
        st = gu.np_state(kf)
        gu.say(f"[lifecycle-batch] member {i} {c.W}x{c.H} new_keyframe {s.new_keyframe}")
        if i == 1:
            assert s.new_keyframe == NEW_KF_INLIERS and np.array_equal(st["x"], c.priors.logdepth.astype(np.float32))
        else:
            assert s.new_keyframe == 0 and not np.array_equal(st["x"], c.priors.logdepth.astype(np.float32))
    batch.close()
