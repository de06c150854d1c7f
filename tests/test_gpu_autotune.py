"""Every autotuner candidate shape solves to oracle parity, and a batch run is
deterministic (two runs bit-identical) -- a race in LDS use or in the team
synchronisation would show as shape- or run-dependent output."""

import numpy as np
import pytest

from gpu_util import dev, map_dtype, np_map_dtype, oracle_semi, rounded_priors, say, torch
from oracle import fusion, stereo
from oracle.fusion import SolverParams
from oracle.stereo import StereoParams
from paper_2207_12244_amd import autotune

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0():
    import kfsynth
    return kfsynth.config_case(0, 0)


def _oracle_state(case):
    sp = StereoParams(n_samples=32, pattern="line5")
    mask = stereo.texture_mask(case.image0)
    z = np.zeros((case.H, case.W))
    r, v, ok, _ = stereo.stereo_update(case.image0, case.images[0], case.K, case.T_wc0, case.poses[0], z, z,
                                       np.zeros((case.H, case.W), bool), mask, sp)
    return np.where(ok, r, 0.0), np.where(ok, v, 0.0)


@pytest.mark.parametrize("threads,ppt", autotune.CANDIDATES)
def test_candidate_shape_parity(c0, threads, ppt):
    from paper_2207_12244_amd.kf import Keyframe
    t = torch()
    tiles = autotune.tiles_for(c0.W, c0.H, threads, ppt)
    say(f"[autotune-shape] {threads}x{ppt} tiles {tiles}")
    rho, var = _oracle_state(c0)
    rho_in, var_in = rho.astype(np.float32), var.astype(np.float32)
    xs = []
    for rep in range(2):
        kf = Keyframe(c0.W, c0.H, precision="bf16", K=c0.K, n_gn=5, n_cg=20, tiles=tiles, solver_threads=threads)
        kf.set_prior(dev(c0.image0, t.uint8), *[dev(m, t.float32) for m in c0.priors.maps()], c0.T_wc0)
        kf.import_state(rho=dev(rho_in, t.float32), var=dev(var_in, t.float32))
        kf.solve()
        xs.append(kf.export_state())
    assert np.array_equal(xs[0]["x"].cpu().numpy(), xs[1]["x"].cpu().numpy()) and xs[0]["tau"] == xs[1]["tau"]
    prior = rounded_priors(c0, "bf16")
    semi = oracle_semi(rho_in.astype(np.float64), var_in.astype(np.float64))
    x_o, tau_o, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=5, n_cg=20, linear_solver="pcg"))
    err = np.abs(xs[0]["x"].cpu().numpy().astype(np.float64) - x_o)
    say(f"[autotune-shape] max|dx| {err.max():.3e} rms {np.sqrt(np.mean(err ** 2)):.3e}")
    assert err.max() <= 2e-4 and np.sqrt(np.mean(err ** 2)) <= 2e-5 and abs(xs[0]["tau"] - tau_o) <= 2e-5


def test_batch_runs_are_deterministic():
    import kfsynth
    from paper_2207_12244_amd.kf import Batch, Keyframe
    t = torch()
    cases = [kfsynth.config_case(3, 40 + i, size_index=i % 4, frames=1) for i in range(6)]
    outs = []
    for rep in range(2):
        members = []
        for c in cases:
            kf = Keyframe(c.W, c.H, K=c.K, precision="bf16", pattern="line5", n_samples=32,
                          tiles=autotune.tiles_for(c.W, c.H, 512, 10), solver_threads=512)
            kf.set_prior(dev(c.image0, t.uint8), *[dev(m, t.float32) for m in c.priors.maps()], c.T_wc0)
            members.append(kf)
        b = Batch(members)
        b.fuse([dev(c.images[0], t.uint8) for c in cases], [c.poses[0] for c in cases])
        outs.append([m.export_state() for m in members])
        b.close()
    for i in range(len(cases)):
        for k in ("x", "rho", "var", "match"):
            assert np.array_equal(outs[0][i][k].cpu().numpy(), outs[1][i][k].cpu().numpy()), (i, k)
        assert outs[0][i]["tau"] == outs[1][i]["tau"]
