"""GPU (gfx950) vs FP64 oracle, stage by stage and end to end, through the C ABI."""

import numpy as np
import pytest

import kfsynth
from oracle import fusion, stereo
from oracle.fusion import SolverParams
from oracle.stereo import StereoParams, UPDATED

import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0():
    return kfsynth.config_case(0, 0)


@pytest.fixture(scope="module")
def c1_short():
    return kfsynth.config_case(1, 0, frames=2)


# ------------------------------------------------------------------ keyframe init

@pytest.mark.parametrize("precision", ["f64", "f32", "bf16"])
def test_prior_init_mask_and_state(c0, precision):
    gu.say(f"[prior-init] config 0 case 0 {precision}")
    kf = gu.make_gpu_kf(c0, precision, "line5", 32)
    st = kf.export_state()
    match = st["match"].cpu().numpy()
    mask = stereo.texture_mask(c0.image0)
    assert np.array_equal(match == -1, mask)                 # texture gate: bit-exact
    assert np.all((match == -1) | (match == -2))
    dt = gu.np_map_dtype(precision)
    assert np.array_equal(st["x"].cpu().numpy(), c0.priors.logdepth.astype(dt))
    assert not st["rho"].cpu().numpy().any() and not st["var"].cpu().numpy().any()
    assert st["tau"] == 0.0
    assert kf.stats().n_searched == int(mask.sum())


# ------------------------------------------------------------------ stereo stage

def _stereo_stage(case, precision, pattern, ns, frames=1):
    """GPU states before and after the stereo update of the last of ``frames``
    frames (earlier frames fused in full), and the FP64 oracle's search from the
    GPU's state before it."""
    t = gu.torch()
    kf = gu.make_gpu_kf(case, precision, pattern, ns)
    for f in range(frames - 1):
        kf.fuse_frame(gu.dev(case.images[f], t.uint8), case.poses[f])
    pre = gu.np_state(kf)
    kf.stereo_update(gu.dev(case.images[frames - 1], t.uint8), case.poses[frames - 1])
    mid = gu.np_state(kf)
    n_upd = kf.stats().n_updated
    sp = StereoParams(n_samples=ns, pattern=pattern)
    res = stereo.epipolar_search(case.image0, case.images[frames - 1], case.K, case.T_wc0, case.poses[frames - 1],
                                 pre["rho"], pre["var"], pre["var"] > 0, stereo.texture_mask(case.image0), sp)
    return pre, mid, res, n_upd


@pytest.mark.parametrize("pattern", ["line5", "sq5x5"])
def test_stereo_first_frame_f64(c0, pattern):
    gu.say(f"[stereo] config 0 case 0 f64 {pattern} N_s=32")
    pre, mid, res, n_upd = _stereo_stage(c0, "f64", pattern, 32)
    P = 5 if pattern == "line5" else 25
    gu.compare_stereo(res, pre, mid, gu.r18_eps("f64", P), (1e-10, 1e-9), f"stereo-f64-{pattern}",
                      max_band_frac=1e-3)
    assert n_upd == int(np.sum(res.status == UPDATED))


@pytest.mark.parametrize("pattern", ["line5", "sq5x5"])
def test_stereo_second_frame_f64(pattern):
    """Second frame: the filter holds estimates, so the search runs over rho +- 2 sqrt(v)
    and the filter takes the Gaussian product (readings R3, R8)."""
    case = kfsynth.config_case(0, 0, frames=2)
    gu.say(f"[stereo] config 0 case 0 f64 {pattern} N_s=32, second frame")
    pre, mid, res, n_upd = _stereo_stage(case, "f64", pattern, 32, frames=2)
    P = 5 if pattern == "line5" else 25
    out = gu.compare_stereo(res, pre, mid, gu.r18_eps("f64", P), (1e-10, 1e-9), f"stereo-f64-{pattern}-frame2",
                            max_band_frac=1e-3)
    assert out["filtered"] > 0.5 * out["compared"]      # the product branch is what is being compared
    assert n_upd == int(np.sum(res.status == UPDATED))


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_stereo_first_frame_sq5x5_float(c1_short, precision):
    """Float kernels against the FP64 oracle: index parity outside the R18 band."""
    c = c1_short
    gu.say(f"[stereo] config 1 case 0 {precision} sq5x5 N_s=64")
    pre, mid, res, n_upd = _stereo_stage(c, precision, "sq5x5", 64)
    gu.compare_stereo(res, pre, mid, gu.r18_eps("f32", 25), (2e-3, 2e-2), f"stereo-{precision}-sq5x5")


@pytest.mark.parametrize("size_index", [1, 3])
@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_stereo_line5_float_batched_sizes(precision, size_index):
    """LINE5, N_s = 32 at the batched workload's sizes (320 x 240, 640 x 480), first
    and second frame. F32: index parity with the FP64 oracle outside the R18 band.
    BF16 rounds the interpolated keyframe points (up to half a grey level), which
    moves SSDs by more than the band: its index mismatch rate against FP64 is
    reported and bounded (<= 5 %; measured 1.6 % at 320 x 240 and 2.8 % at
    640 x 480), and the RMS of the inverse-depth error where the decisions agree
    (<= 2e-2)."""
    case = kfsynth.config_case(3, 0, frames=2, size_index=size_index)
    for frames in (1, 2):
        gu.say(f"[stereo] config 3 {case.W}x{case.H} {precision} line5 N_s=32 frame {frames}")
        pre, mid, res, _ = _stereo_stage(case, precision, "line5", 32, frames=frames)
        label = f"stereo-{precision}-line5-{case.W}x{case.H}-frame{frames}"
        if precision == "f32":
            gu.compare_stereo(res, pre, mid, gu.r18_eps("f32", 5), (2e-3, 2e-2), label)
        else:
            out = gu.compare_stereo(res, pre, mid, gu.r18_eps("f32", 5), None, label, index_parity=False,
                                    value_rms=2e-2)
            assert out["mismatch"] <= 0.05 * out["with_index"], out


# ------------------------------------------------------------------ solver stage

def _oracle_state(case):
    """FP64 oracle filter state after the first frame (the input both solvers get)."""
    sp = StereoParams(n_samples=32, pattern="line5")
    mask = stereo.texture_mask(case.image0)
    z = np.zeros((case.H, case.W))
    r, v, ok, _ = stereo.stereo_update(case.image0, case.images[0], case.K, case.T_wc0, case.poses[0], z, z,
                                       np.zeros((case.H, case.W), bool), mask, sp)
    return np.where(ok, r, 0.0), np.where(ok, v, 0.0)


@pytest.mark.parametrize("precision,mode", [("f64", "rtol"), ("f64", "textbook"), ("f64", "pipelined"),
                                            ("f32", "textbook"), ("f32", "pipelined"), ("bf16", "pipelined")])
def test_solver_parity(c0, precision, mode):
    gu.say(f"[solver] config 0 case 0 {precision} {mode}")
    rho, var = _oracle_state(c0)
    dt = gu.np_map_dtype(precision)
    rho_in, var_in = rho.astype(dt), var.astype(dt)
    if mode == "rtol":
        kf = gu.make_gpu_kf(c0, precision, "line5", 32, n_gn=10, cg_rtol=1e-12, cg_max=4000)
        prm = SolverParams(n_gn=10, cg_rtol=1e-12, cg_max=4000, linear_solver="pcg")
    else:
        kf = gu.make_gpu_kf(c0, precision, "line5", 32, n_gn=10, n_cg=20, cg_variant=mode)
        prm = SolverParams(n_gn=10, n_cg=20, linear_solver="pcg")
    t = gu.torch()
    mdt = gu.map_dtype(precision)
    kf.import_state(rho=gu.dev(rho_in, mdt), var=gu.dev(var_in, mdt))
    kf.solve()
    st = kf.export_state()
    x_gpu = st["x"].cpu().numpy().astype(np.float64)
    prior = gu.rounded_priors(c0, precision)
    semi = gu.oracle_semi(rho_in.astype(np.float64), var_in.astype(np.float64))
    x_o, tau_o, info = fusion.gauss_newton(prior.mu, 0.0, prior, semi, prm)
    err = np.abs(x_gpu - x_o)
    s = kf.stats()
    gu.say(f"[solver-{precision}-{mode}] max|dx| {err.max():.3e} rms {np.sqrt(np.mean(err**2)):.3e} "
           f"dtau {abs(st['tau'] - tau_o):.3e} cg_its {s.cg_iterations} relres {s.cg_rel_residual:.2e} "
           f"n_valid {s.n_valid} (oracle {int(semi.valid.sum())})")
    assert s.n_valid == int(semi.valid.sum())
    if precision == "f64":
        assert err.max() <= 1e-10 and abs(st["tau"] - tau_o) <= 1e-10
        if mode == "rtol":
            # same stopping rule -> same iteration count; the distance to the direct
            # solve is the configured truncation (the oracle's own PCG shows it too)
            assert s.cg_iterations == sum(info.cg_iterations)
            x_d, tau_d, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi,
                                                SolverParams(n_gn=10, linear_solver="direct"))
            e_d = np.abs(x_gpu - x_d).max()
            gu.say(f"[solver-f64-rtol] vs direct solves: max|dx| {e_d:.3e}")
            assert e_d <= 5e-9
    else:
        assert err.max() <= 2e-4 and np.sqrt(np.mean(err ** 2)) <= 2e-5 and abs(st["tau"] - tau_o) <= 2e-5


@pytest.mark.parametrize("precision,threads,tiles,variant", [
    ("f32", 512, (2, 2), "pipelined"), ("f32", 512, (3, 2), "pipelined"), ("f32", 512, (4, 2), "textbook"),
    ("f32", 1024, (4, 2), "pipelined"), ("f32", 256, (4, 3), "pipelined"), ("f64", 256, (4, 4), "pipelined"),
    ("f64", 512, (4, 3), "textbook"), ("f64", 1024, (5, 4), "pipelined"),
    # 160 x 6 tiles: a perimeter of 332 boundary slots, more than the 256 threads that publish them
    ("f32", 256, (1, 20), "pipelined"), ("f64", 256, (1, 20), "textbook")])
def test_solver_tile_shapes(c0, precision, threads, tiles, variant):
    """Every workgroup size and pixels-per-thread class of the solver against the oracle, and tile
    shapes whose boundary has more slots than the workgroup has threads."""
    gu.say(f"[solver-shape] config 0 case 0 {precision} {threads} threads tiles {tiles} {variant}")
    rho, var = _oracle_state(c0)
    dt = gu.np_map_dtype(precision)
    rho_in, var_in = rho.astype(dt), var.astype(dt)
    kf = gu.make_gpu_kf(c0, precision, "line5", 32, n_gn=4, n_cg=20, tiles=tiles, solver_threads=threads,
                        cg_variant=variant)
    lay = kf.solver_layout()
    assert (lay["tiles_x"], lay["tiles_y"], lay["threads"]) == (tiles[0], tiles[1], threads)
    mdt = gu.map_dtype(precision)
    kf.import_state(rho=gu.dev(rho_in, mdt), var=gu.dev(var_in, mdt))
    kf.solve()
    st = kf.export_state()
    prior = gu.rounded_priors(c0, precision)
    semi = gu.oracle_semi(rho_in.astype(np.float64), var_in.astype(np.float64))
    x_o, tau_o, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi,
                                        SolverParams(n_gn=4, n_cg=20, linear_solver="pcg"))
    err = np.abs(st["x"].cpu().numpy().astype(np.float64) - x_o)
    gu.say(f"[solver-shape] max|dx| {err.max():.3e} rms {np.sqrt(np.mean(err ** 2)):.3e} "
           f"dtau {abs(st['tau'] - tau_o):.3e}")
    if precision == "f64":
        assert err.max() <= 1e-10 and abs(st["tau"] - tau_o) <= 1e-10
    else:
        assert err.max() <= 2e-4 and np.sqrt(np.mean(err ** 2)) <= 2e-5 and abs(st["tau"] - tau_o) <= 2e-5


def test_solver_ragged_tiles(c0):
    """Explicit 7 x 5 tiling of 160 x 120 (ragged last column / row of tiles)."""
    gu.say("[solver] config 0 case 0 f64 fixed tiles 7x5")
    rho, var = _oracle_state(c0)
    kf = gu.make_gpu_kf(c0, "f64", "line5", 32, n_gn=3, n_cg=15, tiles=(7, 5))
    t = gu.torch()
    kf.import_state(rho=gu.dev(rho, t.float64), var=gu.dev(var, t.float64))
    kf.solve()
    st = kf.export_state()
    prior = gu.rounded_priors(c0, "f64")
    x_o, tau_o, _ = fusion.gauss_newton(prior.mu, 0.0, prior, gu.oracle_semi(rho, var),
                                        SolverParams(n_gn=3, n_cg=15, linear_solver="pcg"))
    err = np.abs(st["x"].cpu().numpy() - x_o)
    gu.say(f"[solver-ragged] max|dx| {err.max():.3e} dtau {abs(st['tau'] - tau_o):.3e}")
    assert err.max() <= 1e-10 and abs(st["tau"] - tau_o) <= 1e-10


@pytest.mark.parametrize("precision,tiles", [("f64", (54, 4)), ("f64", (14, 18)), ("f32", (54, 4)),
                                             ("f32", (14, 18))])
def test_solver_two_deep_boundary_ragged(c0, precision, tiles):
    """Fixed-count pipelined CG assembles the ghost values of its first stencil
    operand from x shipped two pixels deep (no initial-residual
    synchronisation). 54 x 4 tiles of 160 x 120: tiles 3 px wide, the last
    column 1 px wide (its left neighbour's second ring to the right lies
    outside the image); 14 x 18: tiles 7 px high, the last row 1 px high. Both
    against the oracle's iteration-matched solve."""
    gu.say(f"[solver-2deep] config 0 case 0 {precision} tiles {tiles}")
    rho, var = _oracle_state(c0)
    dt = gu.np_map_dtype(precision)
    rho_in, var_in = rho.astype(dt), var.astype(dt)
    kf = gu.make_gpu_kf(c0, precision, "line5", 32, n_gn=3, n_cg=15, tiles=tiles, solver_threads=256,
                        cg_variant="pipelined")
    mdt = gu.map_dtype(precision)
    kf.import_state(rho=gu.dev(rho_in, mdt), var=gu.dev(var_in, mdt))
    kf.solve()
    s = kf.stats()
    st = kf.export_state()
    prior = gu.rounded_priors(c0, precision)
    semi = gu.oracle_semi(rho_in.astype(np.float64), var_in.astype(np.float64))
    x_o, tau_o, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi,
                                        SolverParams(n_gn=3, n_cg=15, linear_solver="pcg"))
    err = np.abs(st["x"].cpu().numpy().astype(np.float64) - x_o)
    gu.say(f"[solver-2deep] max|dx| {err.max():.3e} rms {np.sqrt(np.mean(err ** 2)):.3e} "
           f"dtau {abs(st['tau'] - tau_o):.3e} syncs {s.team_syncs}")
    assert s.team_syncs == 3 * (15 + 1)   # per GN iteration: the CG iterations and the scale step
    if precision == "f64":
        assert err.max() <= 1e-10 and abs(st["tau"] - tau_o) <= 1e-10
    else:
        assert err.max() <= 2e-4 and np.sqrt(np.mean(err ** 2)) <= 2e-5 and abs(st["tau"] - tau_o) <= 2e-5


def _random_tilings(n, seed=2207):
    """Seeded (W, H, tiles_x, tiles_y) with tiles of at least 2 x 2 px, no empty
    tile, at most 256 tiles and a second ring that fits one slot per thread of a
    256-thread workgroup: the conditions under which the pipelined solve
    assembles its ghost rows from x shipped two pixels deep."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        W, H = int(rng.integers(40, 201)), int(rng.integers(30, 151))
        tx, ty = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        tw, th = -(-W // tx), -(-H // ty)
        if tx * ty > 256 or (tx - 1) * tw >= W or (ty - 1) * th >= H or tw < 2 or th < 2:
            continue
        if 2 * (tw + th) + 4 > 256 or tw * th > 256 * 6:
            continue
        out.append((W, H, tx, ty))
    return out


@pytest.mark.parametrize("W,H,tx,ty", _random_tilings(6))
def test_solver_two_deep_boundary_random_tilings(W, H, tx, ty):
    """The two-deep exchange on seeded random sizes and tilings (ragged last
    rows and columns of tiles included), FP64 pipelined 3 x 15 against the
    oracle's iteration-matched solve."""
    gu.say(f"[solver-2deep-random] {W}x{H} tiles {tx}x{ty} f64")
    case = kfsynth.make_case(7000 + W * 1000 + H, W, H, 1)
    rho, var = _oracle_state(case)
    kf = gu.make_gpu_kf(case, "f64", "line5", 32, n_gn=3, n_cg=15, tiles=(tx, ty), solver_threads=256,
                        cg_variant="pipelined")
    t = gu.torch()
    kf.import_state(rho=gu.dev(rho, t.float64), var=gu.dev(var, t.float64))
    kf.solve()
    s = kf.stats()
    st = kf.export_state()
    prior = gu.rounded_priors(case, "f64")
    x_o, tau_o, _ = fusion.gauss_newton(prior.mu, 0.0, prior, gu.oracle_semi(rho, var),
                                        SolverParams(n_gn=3, n_cg=15, linear_solver="pcg"))
    err = np.abs(st["x"].cpu().numpy() - x_o)
    gu.say(f"[solver-2deep-random] max|dx| {err.max():.3e} dtau {abs(st['tau'] - tau_o):.3e} syncs {s.team_syncs}")
    assert s.team_syncs == 3 * (15 + 1)
    assert err.max() <= 1e-10 and abs(st["tau"] - tau_o) <= 1e-10


def test_prior_only_returns_prior_gpu():
    """P1 on the GPU: texture-free keyframe (S empty) and g = forward difference of mu."""
    case = kfsynth.make_case(77, 96, 64, 1)
    mu = case.priors.logdepth
    gx = np.zeros_like(mu)
    gx[:, :-1] = mu[:, 1:] - mu[:, :-1]
    gy = np.zeros_like(mu)
    gy[:-1, :] = mu[1:, :] - mu[:-1, :]
    maps = (mu, case.priors.logdepth_var, gx, case.priors.gx_var, gy, case.priors.gy_var)
    flat = case.image0.copy()
    flat[:] = 128
    case.image0 = flat
    for precision, tol in (("f64", 1e-12), ("f32", 2e-6)):
        gu.say(f"[prior-only] 96x64 {precision}")
        kf = gu.make_gpu_kf(case, precision, "line5", 32, priors=maps)
        t = gu.torch()
        kf.fuse_frame(gu.dev(case.images[0], t.uint8), case.poses[0])
        d, s = kf.read_depth()
        st = kf.stats()
        assert st.n_searched == 0 and st.n_valid == 0
        x = np.log(d.cpu().numpy().astype(np.float64))
        gu.say(f"[prior-only-{precision}] max|x-mu| {np.abs(x - mu).max():.3e} scale {s}")
        assert np.abs(x - mu.astype(gu.np_map_dtype(precision))).max() <= tol and s == 1.0


def test_pure_rotation_produces_no_measurement(c0):
    gu.say("[rotation] config 0 case 0 f32, zero translation")
    T = c0.poses[0].copy()
    T[:3, 3] = 0.0
    kf = gu.make_gpu_kf(c0, "f32", "line5", 32)
    t = gu.torch()
    kf.stereo_update(gu.dev(c0.images[0], t.uint8), T)
    st = kf.export_state()
    assert not st["var"].cpu().numpy().any()
    assert kf.stats().n_updated == 0


@pytest.mark.parametrize("bad", ["nan_mu", "zero_var", "neg_gvar"])
def test_invalid_prior_reported(c0, bad):
    from paper_2207_12244_amd.kf import KfError, KF_ERR_INPUT
    gu.say(f"[input-error] {bad}")
    mu, vn, gx, vgx, gy, vgy = [m.copy() for m in c0.priors.maps()]
    if bad == "nan_mu":
        mu[5, 7] = np.nan
    elif bad == "zero_var":
        vn[3, 3] = 0.0
    else:
        vgx[9, 9] = -1.0
    kf = gu.make_gpu_kf(c0, "f32", "line5", 32, priors=(mu, vn, gx, vgx, gy, vgy))
    with pytest.raises(KfError) as ei:
        kf.read_depth()
    assert ei.value.status == KF_ERR_INPUT


# ------------------------------------------------------------------ end to end

def test_end_to_end_config0(c0):
    """Plain FP64 form, one frame: stereo + 10 GN iterations (PCG to 1e-12) vs oracle (direct)."""
    gu.say("[e2e] config 0 case 0 f64 line5 N_s=32 rtol 1e-12")
    kf = gu.make_gpu_kf(c0, "f64", "line5", 32, n_gn=10, cg_rtol=1e-12, cg_max=4000)
    t = gu.torch()
    kf.fuse_frame(gu.dev(c0.images[0], t.uint8), c0.poses[0])
    d, s = kf.read_depth()
    st = kf.export_state()
    from oracle import OracleKeyframe
    ok = OracleKeyframe(c0.K, c0.W, c0.H, StereoParams(n_samples=32, pattern="line5"),
                        SolverParams(n_gn=10, cg_rtol=1e-12, cg_max=4000, linear_solver="pcg"))
    ok.set_prior(c0.image0, *c0.priors.maps(), c0.T_wc0)
    rep = ok.fuse_frame(c0.images[0], c0.poses[0])
    res = rep.search
    match = st["match"].cpu().numpy().ravel()[res.pix]
    mism = np.count_nonzero(match != res.k_best)
    d_o, s_o = ok.read_depth()
    err = np.abs(np.log(d.cpu().numpy()) - np.log(d_o))
    gu.say(f"[e2e-c0] index mismatches {mism} max|dlogd| {err.max():.3e} scale {s:.12f} vs {s_o:.12f}")
    assert mism == 0
    assert err.max() <= 1e-10 and abs(np.log(s) - np.log(s_o)) <= 1e-10
    # and the configured PCG tolerance keeps it within 5e-9 of direct solves
    x_d, _, _ = fusion.gauss_newton(ok.prior.mu, 0.0, ok.prior, ok.semi(), SolverParams(n_gn=10, linear_solver="direct"))
    gu.say(f"[e2e-c0] vs direct solves max|dlogd| {np.abs(np.log(d.cpu().numpy()) - x_d).max():.3e}")
    assert np.abs(np.log(d.cpu().numpy()) - x_d).max() <= 5e-9


def test_frame_pipelining_gives_the_same_results(c1_short):
    """pipeline_frames = 1 (solve on a second stream, double-buffered filter
    state, next stereo overlapping the solve) ends bit-identical to one stream,
    with reads in between frames."""
    t = gu.torch()
    case = kfsynth.config_case(1, 0, frames=4)
    outs = []
    for pipe in (False, True):
        from paper_2207_12244_amd.kf import Keyframe
        kf = Keyframe(case.W, case.H, precision="f32", pattern="sq5x5", n_samples=64, n_gn=10, n_cg=20, K=case.K,
                      pipeline_frames=pipe)
        kf.set_prior(gu.dev(case.image0, t.uint8), *[gu.dev(m, t.float32) for m in case.priors.maps()],
                     case.T_wc0)
        imgs = [gu.dev(im, t.uint8) for im in case.images]
        mids = []
        for f in range(4):
            kf.fuse_frame(imgs[f], case.poses[f])
            if f == 1:
                mids.append(kf.export_state())
        st = kf.stats()
        outs.append((kf.export_state(), mids, st.n_updated, st.n_valid))
        gu.say(f"[pipeline={pipe}] n_updated {st.n_updated} n_valid {st.n_valid} scale {st.scale:.6f}")
    (a, ma, ua, va), (b, mb, ub, vb) = outs
    for k in ("x", "rho", "var", "match"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k
        assert np.array_equal(ma[0][k].cpu().numpy(), mb[0][k].cpu().numpy()), k
    assert a["tau"] == b["tau"] and (ua, va) == (ub, vb)
