"""Serving loop on the GPU: each stream's result in the mix equals the same
stream served alone (bit-exact: same tiling and arithmetic), and admission
refuses streams beyond the device-memory budget."""

import numpy as np
import pytest

from gpu_util import dev, say, torch

pytestmark = pytest.mark.gpu

KW = dict(precision="f32", pattern="sq5x5", n_samples=64, n_gn=10, n_cg=20)


def _requests(n_streams, n_req, views=3, rate_hz=400.0):
    from kfsynth.serving import serving_stream
    return [serving_stream(i, n_req, views=views, keyframe_every=12, rate_hz=rate_hz) for i in range(n_streams)]


def test_serving_mix_equals_alone():
    from paper_2207_12244_amd.kf import Keyframe
    from paper_2207_12244_amd.serve import Request, Server
    t = torch()
    streams = _requests(4, 26)
    say(f"serving mix: sizes {[(c.W, c.H) for c, _ in streams]}")
    srv = Server(64 << 30, **KW)
    for c, _ in streams:
        srv.open_stream(c.W, c.H, c.K)
    srv.start()
    for sid, (c, reqs) in enumerate(streams):
        for r in reqs:
            srv.submit(sid, Request(r["kind"], r["t"], r["image"], r["pose"], r.get("priors")))
    stats = srv.run()
    say(f"serving stats {stats}")
    assert stats["frames"] == sum(sum(1 for r in reqs if r["kind"] == "frame") for _, reqs in streams)
    for sid, (c, reqs) in enumerate(streams):
        alone = Keyframe(c.W, c.H, K=c.K, solver_threads=512, **KW)
        for r in reqs:
            if r["kind"] == "keyframe":
                alone.set_prior(dev(r["image"], t.uint8), *[dev(m, t.float32) for m in r["priors"]], r["pose"])
            else:
                alone.fuse_frame(dev(r["image"], t.uint8), r["pose"])
        a, b = alone.export_state(), srv.streams[sid].kf.export_state()
        for k in ("x", "rho", "var", "match"):
            assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), (sid, k)
        assert a["tau"] == b["tau"]
    srv.close()


def test_admission_refuses_over_budget():
    from paper_2207_12244_amd.serve import AdmissionError, Server
    srv = Server(1 << 30, **KW)
    need = srv.stream_bytes(640, 480)
    srv2 = Server(need + need // 2, **KW)
    K = np.array([[512.0, 0, 320], [0, 512.0, 240], [0, 0, 1]])
    srv2.open_stream(640, 480, K)
    with pytest.raises(AdmissionError):
        srv2.open_stream(640, 480, K)
    srv3 = Server(need - 1, **KW)
    with pytest.raises(AdmissionError):
        srv3.open_stream(640, 480, K)
    srv2.close()


def test_streams_admitted_as_memory_frees():
    """Three streams requested under a budget that holds two at a time: the
    third is admitted once an earlier one has finished and released its
    memory, and every stream's result equals the stream served alone."""
    from paper_2207_12244_amd.kf import Keyframe
    from paper_2207_12244_amd.serve import Request, Server
    from kfsynth.serving import serving_stream
    t = torch()
    streams = [serving_stream(i, 8, views=3, keyframe_every=20, rate_hz=200.0) for i in range(3)]
    probe = Server(1 << 40, **KW)
    needs = [probe.stream_bytes(c.W, c.H) for c, _ in streams]
    budget = sorted(needs)[-1] + sorted(needs)[-2] + (1 << 20)     # any two streams plus the batch tables
    srv = Server(budget, keep_results=True, **KW)
    sids = [srv.request_stream(c.W, c.H, c.K, [Request(r["kind"], r["t"], r["image"], r["pose"], r.get("priors"))
                                               for r in reqs]) for c, reqs in streams]
    stats = srv.run()
    say(f"admissions {srv.admissions} closes {srv.closes} stats {stats}")
    assert stats["frames"] == sum(sum(1 for r in reqs if r["kind"] == "frame") for _, reqs in streams)
    admitted_at = dict(srv.admissions)
    closed_at = dict(srv.closes)
    assert max(admitted_at.values()) >= min(closed_at.values())      # the last one waited for a close
    assert srv.used <= budget
    # replay each stream alone and compare with what the served stream ended with
    for (c, reqs), sid in zip(streams, sids):
        alone = Keyframe(c.W, c.H, K=c.K, solver_threads=512, **KW)
        for r in reqs:
            if r["kind"] == "keyframe":
                alone.set_prior(dev(r["image"], t.uint8), *[dev(m, t.float32) for m in r["priors"]], r["pose"])
            else:
                alone.fuse_frame(dev(r["image"], t.uint8), r["pose"])
        a, b = alone.export_state(), srv.results[sid]
        for k in ("x", "rho", "var", "match"):
            assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), (sid, k)
        assert a["tau"] == b["tau"]
    srv.close()
