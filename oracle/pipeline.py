"""Keyframe state and the per-frame update (Sec. II, pipeline prose).

A keyframe is created with the network's predictions (log-depth, log-depth
gradients and their variances). Each later frame runs the semi-dense update
(Sec. II-B) and then re-optimises the keyframe depth (Sec. II-C), warm
starting from the previous frame's (x, tau); the keyframe starts from
(mu, 0).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fusion, stereo
from .fusion import PriorMaps, SemiMeasurements, SolverParams
from .stereo import StereoParams


@dataclass
class FrameReport:
    search: stereo.SearchResult
    gn: fusion.GNInfo
    n_searched: int
    n_updated: int
    n_valid: int


class OracleKeyframe:
    def __init__(self, K, W: int, H: int, stereo_params: StereoParams, solver_params: SolverParams,
                 r_floor: float = 1e-6, stereo_dtype=np.float64):
        self.K = np.asarray(K, dtype=np.float64)
        self.W, self.H = int(W), int(H)
        self.sp = stereo_params
        self.fp = solver_params
        self.r_floor = r_floor
        self.stereo_dtype = stereo_dtype

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

    def stereo_update(self, image1, T_wc1):
        r, v, ok, res = stereo.stereo_update(self.I0, np.asarray(image1, dtype=np.uint8), self.K, self.T_wc0,
                                             T_wc1, self.rho, self.var, self.valid, self.mask, self.sp,
                                             self.stereo_dtype)
        self.rho = np.asarray(r, dtype=np.float64)
        self.var = np.asarray(v, dtype=np.float64)
        self.valid = ok
        return res

    def solve(self):
        x, tau, info = fusion.gauss_newton(self.x, self.tau, self.prior, self.semi(), self.fp)
        self.x, self.tau = x, tau
        return info

    def fuse_frame(self, image1, T_wc1) -> FrameReport:
        res = self.stereo_update(image1, T_wc1)
        info = self.solve()
        return FrameReport(res, info, int(res.pix.size), int(np.sum(res.status == stereo.UPDATED)),
                           int(self.valid.sum()))

    def read_depth(self):
        return np.exp(self.x), float(np.exp(self.tau))
