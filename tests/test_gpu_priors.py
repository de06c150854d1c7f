"""Network outputs at the network's resolution (Sec. II-A; reading R25) ingested on
the GPU (kf_set_prior_network) against the oracle's resampling: the resident
log-depth right after the new keyframe is the resampled, focal-shifted network
log-depth, and a full frame fused from those priors matches the oracle keyframe
built from the oracle's resampled maps."""

import numpy as np
import pytest

import kfsynth
from oracle import OracleKeyframe, SolverParams, StereoParams
from oracle.priors import network_priors, resample_bilinear

import gpu_util as gu

pytestmark = pytest.mark.gpu


def _net_maps(case, Wn=256, Hn=192, focal_ref=None):
    """Stand-in network outputs at Wn x Hn: the case's priors resampled there and
    expressed as the network would give them (log-depth normalised by the focal
    length, gradients per network pixel)."""
    fx = case.K[0, 0]
    sx, sy = Wn / case.W, Hn / case.H
    f_ref = focal_ref if focal_ref is not None else 0.9 * fx * sx
    mu, vmu, gx, vgx, gy, vgy = (resample_bilinear(m, Wn, Hn) for m in case.priors.maps())
    return [mu - np.log(fx * sx / f_ref), vmu, gx / sx, vgx / sx ** 2, gy / sy, vgy / sy ** 2], f_ref


@pytest.mark.parametrize("precision,config,tol", [("f64", 1, 1e-12), ("f32", 2, 3e-6)])
def test_network_priors_resampled_on_the_gpu(precision, config, tol):
    from paper_2207_12244_amd.kf import Keyframe
    t = gu.torch()
    case = kfsynth.config_case(config, 0, frames=1)
    net, f_ref = _net_maps(case)
    gu.say(f"[priors] {case.W}x{case.H} {precision} from 256x192 network maps, f_ref {f_ref:.3f}")
    dt = gu.map_dtype(precision)
    kf = Keyframe(case.W, case.H, precision=precision, pattern="sq5x5", n_samples=64, n_gn=10, n_cg=20, K=case.K,
                  cg_variant="textbook")
    kf.set_prior_network(gu.dev(case.image0, t.uint8), *[gu.dev(m, dt) for m in net], case.T_wc0, f_ref)
    st = gu.np_state(kf)
    pri = network_priors([np.asarray(m, dtype=gu.np_map_dtype(precision)) for m in net], case.W, case.H,
                         case.K[0, 0], f_ref)
    err = np.abs(st["x"] - pri[0]).max()
    gu.say(f"[priors-{precision}] resident log-depth vs oracle resampling: max|dx| {err:.3e}")
    assert err <= tol
    # one frame fused from those priors (config 1: FP64, stereo + 10 x 20 textbook PCG)
    if precision == "f64":
        kf.fuse_frame(gu.dev(case.images[0], t.uint8), case.poses[0])
        st = gu.np_state(kf)
        ok = OracleKeyframe(case.K, case.W, case.H, StereoParams(n_samples=64, pattern="sq5x5"),
                            SolverParams(n_gn=10, n_cg=20, linear_solver="pcg"))
        ok.set_prior(case.image0, *pri, case.T_wc0)
        ok.fuse_frame(case.images[0], case.poses[0])
        e2 = np.abs(st["x"] - ok.x).max()
        gu.say(f"[priors-f64] after one frame: max|dx| {e2:.3e} tau {st['tau']:.12f} vs {ok.tau:.12f}")
        assert e2 <= 1e-10 and abs(st["tau"] - ok.tau) <= 1e-10
    kf.close()


def test_network_priors_reject_bad_sizes():
    from paper_2207_12244_amd.kf import KF_ERR_ARG, Keyframe, KfError
    t = gu.torch()
    case = kfsynth.make_case(11, 64, 48, 1)
    kf = Keyframe(case.W, case.H, precision="f32", pattern="line5", n_samples=32, K=case.K)
    one = t.ones((1, 1), dtype=t.float32, device="cuda")
    with pytest.raises(KfError) as ei:
        kf.set_prior_network(gu.dev(case.image0, t.uint8), one, one, one, one, one, one, case.T_wc0, 100.0)
    assert ei.value.status == KF_ERR_ARG
    kf.close()
