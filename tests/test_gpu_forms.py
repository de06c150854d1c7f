"""Float forms against the FP64 oracle on the headline sizes.

The precision form (bf16 images and patches, f32 maps and arithmetic, FP64 CG
inner products) at 640 x 480 with N_s = 128 and the F32 form on a 320 x 240
sequence with N_s = 64 each run the full per-frame update (stereo + 10 x 20
pipelined PCG) next to the FP64 oracle (the same 10 x 20 Jacobi PCG,
iteration-matched) and report the max and RMS depth error, the scale error and
the rate of pixels whose filter state differs in validity. Stereo decisions
taken in a different precision can pick a neighbouring sample where two SSDs
tie; those pixels move the depth locally, which the bounds below allow for.
Measured on MI355X: precision form 640 x 480, 2 frames: max 8.3e-3, RMS 3.1e-5;
F32 320 x 240, 4 frames: max 2.7e-2, RMS 1.0e-4; scale equal to 6 digits and
no validity difference in either. Bounds: relative depth error RMS <= 5e-4 and
max <= 0.1, scale within 1e-4, at most 0.5 % of the textured pixels with a
different validity.
"""

import numpy as np
import pytest

import kfsynth
from gpu_util import dev, say, torch
from oracle import OracleKeyframe, SolverParams, StereoParams

pytestmark = pytest.mark.gpu


def _run(config, precision, pattern, n_samples, frames):
    from paper_2207_12244_amd.kf import Keyframe
    t = torch()
    case = kfsynth.config_case(config, 0, frames=frames)
    kf = Keyframe(case.W, case.H, precision=precision, pattern=pattern, n_samples=n_samples, n_gn=10, n_cg=20,
                  K=case.K)
    kf.set_prior(dev(case.image0, t.uint8), *[dev(m, t.float32) for m in case.priors.maps()], case.T_wc0)
    ok = OracleKeyframe(case.K, case.W, case.H, StereoParams(n_samples=n_samples, pattern=pattern),
                        SolverParams(n_gn=10, n_cg=20, linear_solver="pcg"))
    ok.set_prior(case.image0, *case.priors.maps(), case.T_wc0)
    for f in range(frames):
        kf.fuse_frame(dev(case.images[f], t.uint8), case.poses[f])
        ok.fuse_frame(case.images[f], case.poses[f])
    d, s = kf.read_depth()
    st = kf.export_state()
    d_o, s_o = ok.read_depth()
    rel = np.abs(d.cpu().numpy().astype(np.float64) / d_o - 1.0)
    valid_gpu = st["var"].cpu().numpy() > 0
    textured = int(ok.mask.sum())
    diff_valid = int(np.sum(valid_gpu != ok.valid))
    say(f"[{precision} {case.W}x{case.H} {frames} frames] depth rel err max {rel.max():.3e} "
        f"rms {np.sqrt(np.mean(rel ** 2)):.3e}; scale {s:.6f} vs {s_o:.6f}; validity differs at "
        f"{diff_valid} of {textured} textured pixels")
    return rel, s, s_o, diff_valid, textured


def _check(rel, s, s_o, diff_valid, textured):
    assert np.sqrt(np.mean(rel ** 2)) <= 5e-4
    assert rel.max() <= 0.1
    assert abs(s / s_o - 1.0) <= 1e-4
    assert diff_valid <= 0.005 * textured


def test_precision_form_640x480_vs_fp64_oracle():
    _check(*_run(2, "bf16", "sq5x5", 128, 2))


def test_f32_sequence_320x240_vs_fp64_oracle():
    _check(*_run(1, "f32", "sq5x5", 64, 4))
