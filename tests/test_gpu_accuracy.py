"""Depth accuracy of the method and its Sec. III variants against the rendered
ground truth of a synthetic scene, by the share of depth values within 10 % of
it (the measure of Sec. III). Properties the paper's ablations lead one to
expect, on the 30-frame 640 x 480 headline sequence (precision form):
- fusing the frames beats the network prior alone by a wide margin;
- the full cost beats the variant without the pairwise (gradient) terms
  (Table III's ablation).
The full-sequence numbers of all variants over three scenes are printed by
bench.py --accuracy."""

import numpy as np
import pytest

import kfsynth

import gpu_util as gu

pytestmark = pytest.mark.gpu


def _within_10(kf, gt):
    d, _ = kf.read_depth()
    rel = np.abs(d.cpu().numpy().astype(np.float64) - gt) / gt
    return 100.0 * float(np.mean(rel < 0.1))


def test_fusion_beats_prior_and_pairwise_terms_help():
    from paper_2207_12244_amd.kf import Keyframe
    t = gu.torch()
    case = kfsynth.config_case(2, 1)
    gt = case.depth0.astype(np.float64)
    img0 = gu.dev(case.image0, t.uint8)
    priors = [gu.dev(m, t.float32) for m in case.priors.maps()]
    frames = [gu.dev(im, t.uint8) for im in case.images]
    pct = {}
    for name, kw in (("prior", None), ("full", {}), ("nopair", dict(variant="no_pairwise"))):
        gu.say(f"[accuracy] config 2 case 1 640x480 bf16 sq5x5 N_s=128 {name}")
        kf = Keyframe(case.W, case.H, precision="bf16", pattern="sq5x5", n_samples=128, n_gn=10, n_cg=20, K=case.K,
                      **(kw or {}))
        kf.set_prior(img0, *priors, case.T_wc0)
        if kw is not None:
            for f, im in enumerate(frames):
                kf.fuse_frame(im, case.poses[f])
        pct[name] = _within_10(kf, gt)
        kf.close()
    gu.say(f"[accuracy] within 10 %: {pct}")
    assert pct["full"] >= pct["prior"] + 10.0
    assert pct["full"] > pct["nopair"]
