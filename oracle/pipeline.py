"""Keyframe state and the per-frame update (Sec. II, pipeline prose).

A keyframe is created with the network's predictions (log-depth, log-depth
gradients and their variances). Each later frame runs the semi-dense update
(Sec. II-B) and then re-optimises the keyframe depth (Sec. II-C), warm
starting from the previous frame's (x, tau); the keyframe starts from
(mu, 0).

The search of one pixel reads only the two images, the pose and that pixel's
filter state, so it may run on disjoint sets of pixels in separate processes
(``pool``): the rows of the texture mask are cut into contiguous blocks, each
block is searched by the same ``stereo.epipolar_search`` on the whole images,
and the per-pixel results are concatenated back in row-major order. Every
number is the one the single-process call gives; only the wall time changes.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fusion, stereo
from .fusion import PriorMaps, SemiMeasurements, SolverParams
from .stereo import StereoParams


def camera_translation(T_wc0, T_wc1) -> float:
    """Distance between the keyframe's and the new frame's camera centres (the
    translation part of T_wc0^-1 T_wc1, whose norm the rotation leaves unchanged)."""
    c0 = np.asarray(T_wc0, dtype=np.float64)[:3, 3]
    c1 = np.asarray(T_wc1, dtype=np.float64)[:3, 3]
    return float(np.linalg.norm(c1 - c0))


# reasons for a new keyframe (bit flags)
NEW_KF_TRANSLATION = 1
NEW_KF_INLIERS = 2


def keyframe_decision(translation: float, inliers: int, lambda_trans: float = 0.0, lambda_inliers: int = 0) -> int:
    """Sec. II: a new keyframe is created when the camera has translated more
    than lambda_trans or the semi-dense estimation had fewer than lambda_inliers
    inliers (measurements produced by the search). A threshold of 0 disables its
    test. Returns the reason bits (0: keep the keyframe and fuse the frame)."""
    r = 0
    if lambda_trans > 0.0 and translation > lambda_trans:
        r |= NEW_KF_TRANSLATION
    if lambda_inliers > 0 and inliers < lambda_inliers:
        r |= NEW_KF_INLIERS
    return r


def _search_block(args):
    return stereo.epipolar_search(*args)


def merge_search_results(parts) -> stereo.SearchResult:
    """Concatenates the results of row blocks searched in row-major order."""
    fields = stereo.SearchResult.__dataclass_fields__
    return stereo.SearchResult(**{f: np.concatenate([getattr(p, f) for p in parts]) for f in fields})


def search_in_blocks(pool, n_blocks, I0, I1, K, T_wc0, T_wc1, rho, var, valid, mask, params, dtype=np.float64):
    """``stereo.epipolar_search`` over the mask cut into ``n_blocks`` row blocks,
    run by ``pool`` (anything with an order-preserving ``map``)."""
    mask = np.asarray(mask, dtype=bool)
    H = mask.shape[0]
    rows = np.cumsum(mask.sum(axis=1))
    total = int(rows[-1]) if H else 0
    cuts = [0]
    for b in range(1, n_blocks):
        cuts.append(int(np.searchsorted(rows, total * b / n_blocks)))
    cuts.append(H)
    jobs = []
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        if r1 <= r0:
            continue
        m = np.zeros_like(mask)
        m[r0:r1] = mask[r0:r1]
        jobs.append((I0, I1, K, T_wc0, T_wc1, rho, var, valid, m, params, dtype))
    return merge_search_results(list(pool.map(_search_block, jobs)))


@dataclass
class FrameReport:
    search: stereo.SearchResult
    gn: fusion.GNInfo
    n_searched: int
    n_updated: int
    n_valid: int
    new_keyframe: int = 0     # reason bits of keyframe_decision (0: the frame was fused)


class OracleKeyframe:
    def __init__(self, K, W: int, H: int, stereo_params: StereoParams, solver_params: SolverParams,
                 r_floor: float = 1e-6, stereo_dtype=np.float64, pool=None, n_blocks: int = 0,
                 lambda_trans: float = 0.0, lambda_inliers: int = 0):
        self.K = np.asarray(K, dtype=np.float64)
        self.W, self.H = int(W), int(H)
        self.sp = stereo_params
        self.fp = solver_params
        self.r_floor = r_floor
        self.stereo_dtype = stereo_dtype
        self.pool = pool                      # optional process pool for the per-pixel search
        self.n_blocks = n_blocks or 8
        self.lambda_trans = float(lambda_trans)
        self.lambda_inliers = int(lambda_inliers)

    def set_prior(self, image0, mu, var_n, gx, var_gx, gy, var_gy, T_wc0):
        self.I0 = np.asarray(image0, dtype=np.uint8)
        self.prior = PriorMaps(*(np.asarray(a, dtype=np.float64) for a in (mu, var_n, gx, var_gx, gy, var_gy)))
        self.T_wc0 = np.asarray(T_wc0, dtype=np.float64)
        self.mask = stereo.texture_mask(self.I0, self.sp.grad_gate, self.sp.border)
        self.x = self.prior.mu.copy()
        self.tau = 0.0
        self.rho = np.zeros((self.H, self.W))
        self.var = np.zeros((self.H, self.W))
        self.valid = np.zeros((self.H, self.W), dtype=bool)

    def set_state(self, x=None, tau=None, rho=None, var=None, valid=None):
        if x is not None:
            self.x = np.array(x, dtype=np.float64)
        if tau is not None:
            self.tau = float(tau)
        if rho is not None:
            self.rho = np.array(rho, dtype=np.float64)
        if var is not None:
            self.var = np.array(var, dtype=np.float64)
        if valid is not None:
            self.valid = np.array(valid, dtype=bool)

    def semi(self) -> SemiMeasurements:
        z, R, ok = stereo.log_measurements(self.rho, self.var, self.valid, self.r_floor)
        return SemiMeasurements(z, R, ok)

    def search(self, image1, T_wc1) -> stereo.SearchResult:
        """The epipolar search of every textured pixel from the current filter state."""
        args = (self.I0, np.asarray(image1, dtype=np.uint8), self.K, self.T_wc0, T_wc1, self.rho, self.var,
                self.valid, self.mask, self.sp, self.stereo_dtype)
        if self.pool is None:
            return stereo.epipolar_search(*args)
        return search_in_blocks(self.pool, self.n_blocks, *args)

    def stereo_update(self, image1, T_wc1):
        res = self.search(image1, T_wc1)
        upd = res.status == stereo.UPDATED
        dt = np.dtype(self.stereo_dtype)
        r, v, ok = stereo.filter_update(np.asarray(self.rho, dtype=dt), np.asarray(self.var, dtype=dt), self.valid,
                                        res.pix[upd], res.rho_obs[upd], res.var_obs[upd])
        self.rho = np.asarray(r, dtype=np.float64)
        self.var = np.asarray(v, dtype=np.float64)
        self.valid = ok
        return res

    def solve(self):
        x, tau, info = fusion.gauss_newton(self.x, self.tau, self.prior, self.semi(), self.fp)
        self.x, self.tau = x, tau
        return info

    def fuse_frame(self, image1, T_wc1) -> FrameReport:
        """Sec. II per frame: the semi-dense update, then either the fusion or,
        when keyframe_decision asks for a new keyframe, nothing more (the
        keyframe's depth map keeps its last fused state; the caller creates the
        new keyframe with set_prior)."""
        res = self.stereo_update(image1, T_wc1)
        n_upd = int(np.sum(res.status == stereo.UPDATED))
        reason = keyframe_decision(camera_translation(self.T_wc0, T_wc1), n_upd, self.lambda_trans,
                                   self.lambda_inliers)
        info = self.solve() if reason == 0 else fusion.GNInfo()
        return FrameReport(res, info, int(res.pix.size), n_upd, int(self.valid.sum()), reason)

    def read_depth(self):
        return np.exp(self.x), float(np.exp(self.tau))
