"""Batched form on the GPU: every keyframe of a mixed batch ends bit-identical
to the same keyframe fused alone (same tiling, same arithmetic), with and
without graph replay, and when there are more solver teams than co-resident
workgroups so that workgroups run several teams in turn."""

import numpy as np
import pytest

import kfsynth
from gpu_util import dev, map_dtype, say, torch

pytestmark = pytest.mark.gpu

BATCH_KW = dict(precision="bf16", pattern="line5", n_samples=32, n_gn=10, solver_threads=512)


def _make(case, n_cg=20, tiles=(0, 0)):
    from paper_2207_12244_amd.kf import Keyframe
    t = torch()
    kf = Keyframe(case.W, case.H, K=case.K, n_cg=n_cg, tiles=tiles, **BATCH_KW)
    dt = map_dtype(BATCH_KW["precision"])
    kf.set_prior(dev(case.image0, t.uint8), *[dev(m, dt) for m in case.priors.maps()], case.T_wc0)
    return kf


def _state(kf):
    s = kf.export_state()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in s.items()}


def _assert_same(a, b, label):
    for k in ("x", "rho", "var", "match"):
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{label}: {k} differs " \
            f"(max |d| {np.nanmax(np.abs(a[k].astype(np.float64) - b[k].astype(np.float64)))})"
    assert a["tau"] == b["tau"], label


def _run_pair(cases, settings, frames, mode):
    from paper_2207_12244_amd.kf import Batch
    t = torch()
    solo = [_make(c, **s) for c, s in zip(cases, settings)]
    members = [_make(c, **s) for c, s in zip(cases, settings)]
    batch = Batch(members, use_graph=mode != "direct")
    imgs = [[dev(c.images[f], t.uint8) for c in cases] for f in range(frames)]
    for f in range(frames):
        for i, (k, c) in enumerate(zip(solo, cases)):
            k.fuse_frame(imgs[f][i], c.poses[f])
        poses = [c.poses[f] for c in cases]
        if mode == "split":
            batch.stereo_update(imgs[f], poses)
            batch.solve()
        else:
            batch.fuse(imgs[f], poses)
    t.cuda.synchronize()
    return solo, members, batch


@pytest.mark.parametrize("mode", ["graph", "direct", "split"])
def test_batch_equals_solo_mixed_sizes(mode):
    # sizes of the batched workload plus a ragged one; one member with another CG count
    sizes = [0, 1, 2, 3, 0, 1]
    cases = [kfsynth.config_case(3, i, size_index=s, frames=2) for i, s in enumerate(sizes)]
    extra = kfsynth.make_case(kfsynth.seed_for(3, 99), 200, 130, 2, "single")
    cases.append(extra)
    settings = [dict() for _ in cases]
    settings[4] = dict(n_cg=7)
    say(f"batch mixed: sizes {[(c.W, c.H) for c in cases]}, mode={mode}")
    solo, members, batch = _run_pair(cases, settings, 2, mode)
    lay = batch.layout()
    say(f"batch layout {lay}")
    for i, (a, b) in enumerate(zip(solo, members)):
        sa, sb = _state(a), _state(b)
        assert b.stats().n_updated == a.stats().n_updated
        _assert_same(sa, sb, f"member {i} ({cases[i].W}x{cases[i].H})")
        assert np.isfinite(sa["x"]).all()
    batch.close()


def test_batch_queues_more_teams_than_resident_workgroups():
    # 256-workgroup teams (16 x 16 tiles of 320 x 240): more teams than fit at once
    n = 8
    cases = [kfsynth.config_case(3, 10 + i, size_index=1, frames=1) for i in range(n)]
    settings = [dict(tiles=(16, 16)) for _ in cases]
    say(f"batch queued: {n} x 320x240 with 16x16 tiles")
    solo, members, batch = _run_pair(cases, settings, 1, "graph")
    lay = batch.layout()
    say(f"batch layout {lay}")
    assert lay["max_queue"] >= 2, lay
    for i, (a, b) in enumerate(zip(solo, members)):
        _assert_same(_state(a), _state(b), f"member {i}")
    batch.close()


def test_batch_subset_calls_equal_solo():
    """kf_batch_fuse_subset: listed members advance exactly as alone; the rest stay untouched."""
    from paper_2207_12244_amd.kf import Batch
    t = torch()
    cases = [kfsynth.config_case(3, 60 + i, size_index=i % 4, frames=3) for i in range(5)]
    solo = [_make(c) for c in cases]
    members = [_make(c) for c in cases]
    batch = Batch(members)
    plan = [[0, 1, 2, 3, 4], [0, 2, 4], [3, 1]]
    say(f"batch subset: plan {plan}")
    for f, active in enumerate(plan):
        imgs = [dev(cases[i].images[f], t.uint8) for i in active]
        poses = [cases[i].poses[f] for i in active]
        for k, i in enumerate(active):
            solo[i].fuse_frame(imgs[k], poses[k])
        batch.fuse_subset(active, imgs, poses)
    t.cuda.synchronize()
    for i in range(len(cases)):
        _assert_same(_state(solo[i]), _state(members[i]), f"member {i}")
    batch.close()


def test_batch_schedule_fills_the_workgroups():
    """The batched workload's 64-keyframe mix at 512 threads x 10 px per thread
    (14 x 160x120, 22 x 320x240, 16 x 512x384, 12 x 640x480: 4 / 15 / 39 / 60
    tiles) puts 1,730 team members on 256 workgroups. The host places next the
    team that can start earliest, so small teams fill the workgroups that large
    ones would leave waiting, and the longest queue holds ceil(1730 / 256) = 7
    teams (placing the teams in order of decreasing cost left gaps: 8)."""
    from paper_2207_12244_amd.autotune import tiles_for
    from paper_2207_12244_amd.kf import Batch, Keyframe
    t = torch()
    if t.cuda.get_device_properties(0).multi_processor_count != 256:
        pytest.skip("the expected queue length is for a 256-CU device")
    mix = {(160, 120): 14, (320, 240): 22, (512, 384): 16, (640, 480): 12}
    members, total = [], 0
    for (W, H), n in mix.items():
        tx, ty = tiles_for(W, H, 512, 10)
        K = np.array([[0.8 * W, 0.0, W / 2.0], [0.0, 0.8 * W, H / 2.0], [0.0, 0.0, 1.0]])
        for _ in range(n):
            members.append(Keyframe(W, H, K=K, tiles=(tx, ty), **BATCH_KW))
        total += n * tx * ty
    batch = Batch(members, use_graph=False)
    lay = batch.layout()
    say(f"schedule of the 64-keyframe mix: {total} team members, layout {lay}")
    assert total == 1730
    assert lay["workgroups"] == 256 and lay["ppt"] == 10, lay
    assert lay["max_queue"] == -(-total // 256), lay
    batch.close()
    for m in members:
        m.close()
