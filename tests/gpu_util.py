"""Helpers shared by the GPU tests: seeded inputs on the device, matching oracle runs."""

from __future__ import annotations

import sys

import numpy as np

import kfsynth
from oracle import fusion, stereo
from oracle.fusion import PriorMaps, SemiMeasurements, SolverParams
from oracle.stereo import StereoParams


def torch():
    import torch as _t
    return _t


def dev(a, dtype):
    t = torch()
    return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def map_dtype(precision):
    t = torch()
    return t.float64 if precision == "f64" else t.float32


def np_map_dtype(precision):
    return np.float64 if precision == "f64" else np.float32


def make_gpu_kf(case, precision, pattern, n_samples, n_gn=10, n_cg=20, cg_rtol=0.0, cg_max=4000,
                tiles=(0, 0), huber_delta=1.345, priors=None, cg_variant="auto", solver_threads=0):
    from paper_2207_12244_amd.kf import Keyframe
    kf = Keyframe(case.W, case.H, precision=precision, pattern=pattern, n_samples=n_samples, n_gn=n_gn,
                  n_cg=n_cg, cg_rtol=cg_rtol, cg_max=cg_max, K=case.K, tiles=tiles, huber_delta=huber_delta,
                  cg_variant=cg_variant, solver_threads=solver_threads)
    t = torch()
    dt = map_dtype(precision)
    maps = priors if priors is not None else case.priors.maps()
    kf.set_prior(dev(case.image0, t.uint8), *[dev(m, dt) for m in maps], case.T_wc0)
    return kf


def rounded_priors(case, precision):
    """The priors as the GPU form stores them (float32 forms round once), back in float64."""
    dt = np_map_dtype(precision)
    return PriorMaps(*[np.asarray(m, dtype=dt).astype(np.float64) for m in case.priors.maps()])


def oracle_semi(rho, var, r_floor=1e-6):
    valid = var > 0
    z, R, ok = stereo.log_measurements(rho, var, valid, r_floor)
    return SemiMeasurements(z, R, ok)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def first_frame_search(case, pattern, n_samples, dtype=np.float64, mask=None):
    sp = StereoParams(n_samples=n_samples, pattern=pattern)
    m = stereo.texture_mask(case.image0) if mask is None else mask
    z = np.zeros((case.H, case.W))
    return stereo.epipolar_search(case.image0, case.images[0], case.K, case.T_wc0, case.poses[0], z, z,
                                  np.zeros((case.H, case.W), bool), m, sp, dtype)


# ------------------------------------------------------------------ staged comparisons

def np_state(kf):
    """The context's resident state as float64 / int32 numpy arrays (plus tau)."""
    st = kf.export_state()
    out = {k: st[k].cpu().numpy() for k in ("x", "rho", "var", "match")}
    for k in ("x", "rho", "var"):
        out[k] = out[k].astype(np.float64)
    out["tau"] = float(st["tau"])
    return out


def r18_eps(kind, P):
    """Near-tie band of two SSDs b <= s2 (reading R18), eps(b, s2).

    FP64: 1e-9 (1 + b). Float32: 1e-3 (1 + b) + 0.05 P + 0.05 sqrt(P s2). The
    last term bounds what float32 sample coordinates do to an SSD: image
    coordinates up to ~640 carry ~1e-4 px of rounding (a few half-ulps of 640),
    and a shift dp changes SSD = sum_j e_j^2 by at most 2 dp max|grad I| sum_j |e_j|
    <= 2 x 1e-4 x 255 x sqrt(P SSD) (uint8 images: |grad I| <= 255 per px)."""
    if kind == "f64":
        return lambda b, s2=None: 1e-9 * (1.0 + b)
    return lambda b, s2: 1e-3 * (1.0 + b) + 0.05 * P + 0.05 * np.sqrt(P * np.where(np.isfinite(s2), s2, 0.0))


def process_pool(workers=8):
    """Processes for the oracle's per-pixel search (spawned: they never touch the GPU)."""
    import concurrent.futures
    import multiprocessing
    return concurrent.futures.ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("spawn"))


def compare_stereo(res, pre, mid, eps, rel_tol, label, max_band_frac=0.005, index_parity=True,
                   value_rms=None):
    """One stereo update of the GPU (state ``pre`` -> ``mid``) against the oracle's
    search ``res`` from the same state ``pre``.

    Decisions that floating point takes (reading R18) and where either answer
    is correct go to the band:
      - argmin ties: the oracle's two best SSDs within eps(best, second);
      - validity ties: a validity test of the oracle's or the GPU's chosen
        sample is within rounding of its boundary: a tap within 1e-3 px of the
        image edge, or the inverse depth within 1e-5 (relative) of rho_min or
        rho_max (the end samples of an interval clamped to the range sit on the
        bound by construction).
    Outside the band the indices must agree; inside it the GPU takes the other
    index in at most ``max_band_frac`` of the pixels with an index, and an
    argmin-tie choice must be one of the near-best samples. Where the indices
    agree, the decision is clear and the neighbour choice (the lower-SSD of
    k*-1, k*+1) is too: the same update decision, and the filter result (first
    observation, or the Gaussian product with the state ``pre``) within
    ``rel_tol`` = (rho, var) relative, RMS of rho within ``value_rms`` if given.
    Pixels left alone keep ``pre`` exactly. With ``index_parity`` False (BF16
    rounding on the search path) the mismatch rate is only returned."""
    pix = res.pix
    n, NS = res.ssd.shape
    rows = np.arange(n)
    match = mid["match"].ravel()[pix]
    has = res.k_best >= 0
    ssd = np.where(np.isfinite(res.ssd), res.ssd, np.inf)
    s = np.sort(ssd, axis=1)
    best = s[:, 0]
    with np.errstate(invalid="ignore"):
        margin = np.where(np.isfinite(s[:, 1]), s[:, 1] - s[:, 0], np.inf)
    def vtie(k):
        kk = np.clip(k, 0, NS - 1)
        tm, rm = res.tap_margin[rows, kk], res.range_margin[rows, kk]
        return (k >= 0) & (k < NS) & ((np.abs(tm) <= 1e-3) | (np.abs(rm) <= 1e-5))

    tie_v = vtie(res.k_best) | vtie(match)
    with np.errstate(invalid="ignore"):
        band = tie_v | (has & (margin < eps(best, s[:, 1])))
    clear = has & ~band
    mism = match != res.k_best
    out = {"searched": int(n), "with_index": int(has.sum()), "band": int(band.sum()),
           "validity_ties": int(tie_v.sum()),
           "mismatch_clear": int(np.count_nonzero(mism & clear)), "mismatch_band": int(np.count_nonzero(mism & band)),
           "mismatch": int(np.count_nonzero(mism))}
    for r in np.flatnonzero(mism & clear)[:8]:
        k, ko = int(match[r]), int(res.k_best[r])
        say(f"[{label}] clear mismatch at pixel {int(pix[r])}: oracle k {ko} ssd {ssd[r, ko]:.4f}, gpu k {k} ssd "
            f"{ssd[r, k] if k >= 0 else float('nan'):.4f}, second {s[r, 1]:.4f} eps {float(eps(best[r], s[r, 1])):.4f} "
            f"rho_k {res.rho_k[r, ko]:.6f}")
    if index_parity:
        assert out["mismatch_clear"] == 0, f"[{label}] {out['mismatch_clear']} index mismatches outside the band: {out}"
        assert out["mismatch_band"] <= max_band_frac * max(1, out["with_index"]), f"[{label}] band choices {out}"
        for r in np.flatnonzero(band & mism & ~tie_v):
            k = match[r]
            assert k >= 0 and ssd[r, k] <= best[r] + eps(best[r], ssd[r, k]), (label, r, k)
        none = ~has & ~tie_v
        assert np.array_equal(match[none], np.full(none.sum(), -1))
    # neighbour choice of the oracle: lower SSD of k*-1 and k*+1 (tie -> k*-1)
    kb = np.clip(res.k_best, 0, NS - 1)
    s_m = np.where(res.k_best - 1 >= 0, ssd[rows, np.clip(res.k_best - 1, 0, NS - 1)], np.inf)
    s_p = np.where(res.k_best + 1 < NS, ssd[rows, np.clip(res.k_best + 1, 0, NS - 1)], np.inf)
    with np.errstate(invalid="ignore"):
        tie_n = (np.isfinite(s_m) & np.isfinite(s_p)
                 & (np.abs(s_m - s_p) < eps(np.minimum(s_m, s_p), np.maximum(s_m, s_p)))) \
            | vtie(res.k_best - 1) | vtie(res.k_best + 1)
    cmp = ~mism & clear & ~tie_n
    upd = res.status == stereo.UPDATED
    pre_valid = pre["var"].ravel()[pix] > 0
    rho_mid = mid["rho"].ravel()[pix]
    var_mid = mid["var"].ravel()[pix]
    moved = (rho_mid != pre["rho"].ravel()[pix]) | (var_mid != pre["var"].ravel()[pix])
    out["neighbour_ties"] = int(np.count_nonzero(~mism & clear & tie_n))
    out["update_decision_differs"] = int(np.count_nonzero(cmp & (upd != moved)))
    if index_parity:
        assert out["update_decision_differs"] == 0, f"[{label}] update decisions differ: {out}"
    same = cmp & upd & moved
    rp, vp = pre["rho"].ravel()[pix][same], pre["var"].ravel()[pix][same]
    ro, vo = res.rho_obs[same], res.var_obs[same]
    pv = pre_valid[same]
    exp_r = np.where(pv, (vo * rp + vp * ro) / np.where(pv, vp + vo, 1.0), ro)
    exp_v = np.where(pv, vp * vo / np.where(pv, vp + vo, 1.0), vo)
    er = np.abs(rho_mid[same] / exp_r - 1.0)
    ev = np.abs(var_mid[same] / exp_v - 1.0)
    out.update(compared=int(same.sum()), filtered=int(np.count_nonzero(pv)),
               rho_rel_max=float(er.max()) if er.size else 0.0,
               rho_rel_rms=float(np.sqrt(np.mean(er ** 2))) if er.size else 0.0,
               var_rel_max=float(ev.max()) if ev.size else 0.0)
    say(f"[{label}] {out}")
    if rel_tol is not None:
        assert out["rho_rel_max"] <= rel_tol[0] and out["var_rel_max"] <= rel_tol[1], f"[{label}] filter values {out}"
    if value_rms is not None:
        assert out["rho_rel_rms"] <= value_rms, f"[{label}] filter values {out}"
    return out


def oracle_solve_from(pre_x, pre_tau, prior, mid, n_gn, n_cg):
    """Iteration-matched FP64 oracle solve (Jacobi PCG, n_gn x n_cg) from the GPU's
    own state: x and tau before the solve, filter state after the stereo update."""
    semi = oracle_semi(mid["rho"], mid["var"])
    x_o, tau_o, _ = fusion.gauss_newton(pre_x, pre_tau, prior, semi,
                                        SolverParams(n_gn=n_gn, n_cg=n_cg, linear_solver="pcg"))
    return x_o, tau_o, semi
