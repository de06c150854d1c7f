"""Seeded request streams for the serving workload: per camera stream, a
keyframe case rendered at a few views, and a Poisson arrival process.

A stream's input is a sequence of requests in arrival order. Every
`keyframe_every`-th request is a new keyframe (its image, the six prior maps
and its pose, as the network would deliver them); the others are new frames
that cycle back and forth through the rendered views (a camera moving along
its path and back), so long streams need only a few rendered images. Each new
keyframe after the first carries freshly drawn network priors (the same
noise model around the true log-depth, new seeded draws), stored as float32.
"""

from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .scene import CONFIGS, KeyframeCase, config_case, make_priors, seed_for


def serving_stream(stream: int, n_requests: int, views: int = 4, keyframe_every: int = 20,
                   rate_hz: float = None, config: int = 4) -> Tuple[KeyframeCase, List[dict]]:
    cfg = CONFIGS[config]
    rate = cfg.get("rate_hz", 30.0) if rate_hz is None else rate_hz
    case = config_case(config, stream, frames=views)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_for(config, stream), 11])))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    # view order 0, 1, .., V-1, V-2, .., 1, 0, 1, ...
    cycle = list(range(views)) + list(range(views - 2, 0, -1)) if views > 1 else [0]
    reqs, k = [], 0
    for i in range(n_requests):
        if i % keyframe_every == 0:
            j = i // keyframe_every
            if j == 0:
                pri = case.priors.maps()
            else:
                prng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_for(config, stream), 13, j])))
                pri = tuple(m.astype(np.float32) for m in make_priors(prng, case.depth0).maps())
            reqs.append(dict(kind="keyframe", t=float(t[i]), image=case.image0, pose=case.T_wc0, priors=pri))
            k = 0
        else:
            v = cycle[k % len(cycle)]
            k += 1
            reqs.append(dict(kind="frame", t=float(t[i]), image=case.images[v], pose=case.poses[v]))
    return case, reqs
