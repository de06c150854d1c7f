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
