"""Shape autotuner for the batched solver.

A batch runs every member's solver team inside one persistent launch, so its
throughput depends on how many pixels each co-resident workgroup holds (more
pixels per workgroup amortise the team synchronisations, fewer keep more
teams in flight). The tuner times the candidate policies -- a workgroup size
and a cap on pixels per thread, from which each member's tile grid follows --
on a throw-away batch of the requested sizes (a flat image and seeded random
priors: at a fixed iteration count the solver's run time does not depend on
the data, as long as the residual is not zero) and caches the winner in a
JSON file keyed by device, form and size mix.

    from paper_2207_12244_amd import autotune
    pol = autotune.tuned_policy([(640, 480), (160, 120)], precision="bf16")
    tiles = autotune.tiles_for(640, 480, pol["threads"], pol["ppt"])
"""

from __future__ import annotations

import json
import os
import time
from typing import Iterable, Optional, Sequence, Tuple

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")
CANDIDATES = ((512, 10), (512, 8), (512, 6), (1024, 3), (512, 4), (512, 3))
MAX_TEAM = 256


def tiles_for(W: int, H: int, threads: int, ppt: int) -> Optional[Tuple[int, int]]:
    """The tile grid with the fewest tiles of at most threads * ppt pixels
    (ties: the shortest tile perimeter), within the library's tiling rules."""
    cap = threads * ppt
    best = None
    for tx in range(1, min(64, W) + 1):
        tw = -(-W // tx)
        if (tx - 1) * tw >= W:
            continue
        for ty in range(1, min(64, H) + 1):
            th = -(-H // ty)
            if tx * ty > MAX_TEAM or (ty - 1) * th >= H or tw * th > cap or tw + th > threads:
                continue
            key = (tx * ty, tw + th)
            if best is None or key < best[0]:
                best = (key, (tx, ty))
    return best[1] if best else None


def cache_key(sizes: Iterable[Tuple[int, int]], precision: str, n_gn: int, n_cg: int, device: str) -> str:
    mix = {}
    for W, H in sizes:
        mix[f"{W}x{H}"] = mix.get(f"{W}x{H}", 0) + 1
    mix_s = ",".join(f"{k}:{mix[k]}" for k in sorted(mix))
    return f"{device}|{precision}|gn{n_gn}|cg{n_cg}|{mix_s}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _device_name() -> str:
    """Architecture and compute-unit count of device 0, e.g. "gfx950-256cu"."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}-{p.multi_processor_count}cu".replace("|", "/")


def measure_policy(sizes: Sequence[Tuple[int, int]], threads: int, ppt: int, precision: str = "bf16",
                   n_gn: int = 10, n_cg: int = 20, reps: int = 4) -> Optional[float]:
    """Fastest of `reps` timed solves (after two untimed ones) of one batch of
    the given sizes under a policy, in milliseconds, or None if the policy
    does not fit (no tiling, or a team cannot be co-resident)."""
    import numpy as np
    import torch
    from .kf import Batch, Keyframe, KfError
    members = []
    dt = torch.float64 if precision == "f64" else torch.float32
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12244)
    try:
        for W, H in sizes:
            tiles = tiles_for(W, H, threads, ppt)
            if tiles is None:
                return None
            kf = Keyframe(W, H, precision=precision, n_gn=n_gn, n_cg=n_cg, tiles=tiles, solver_threads=threads)
            # flat image (no stereo work) and random priors: a nonzero residual
            # keeps every CG iteration running
            img = torch.full((H, W), 128, dtype=torch.uint8, device="cuda")
            maps = [torch.rand((H, W), generator=gen, dtype=dt, device="cuda") for _ in range(3)]
            var = torch.full((H, W), 0.01, dtype=dt, device="cuda")
            kf.set_prior(img, maps[0], var, maps[1], var, maps[2], var, np.eye(4))
            members.append(kf)
        b = Batch(members)
    except KfError:
        return None
    stream = members[0].stream
    b.solve()
    b.solve()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        b.solve()
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.min([e0.elapsed_time(e1) for e0, e1 in ev]))
    b.close()
    return ms


def tune(sizes: Sequence[Tuple[int, int]], precision: str = "bf16", n_gn: int = 10, n_cg: int = 20,
         candidates=CANDIDATES, cache: Optional[str] = None, verbose: bool = False) -> dict:
    """Times every candidate policy on the size mix (two rounds, so that clock
    ramp-up does not favour the later candidates) and records the fastest."""
    path = cache or os.environ.get("KF_TUNE_CACHE") or DEFAULT_CACHE
    best = {}
    for rnd in range(2):
        for threads, ppt in candidates:
            t0 = time.perf_counter()
            ms = measure_policy(sizes, threads, ppt, precision, n_gn, n_cg)
            if verbose:
                print(f"# autotune round {rnd} {threads}x{ppt}: {ms} ms ({time.perf_counter() - t0:.1f}s)", flush=True)
            if ms is not None:
                best[(threads, ppt)] = min(ms, best.get((threads, ppt), ms))
    results = [(ms, t, p) for (t, p), ms in best.items()]
    if not results:
        raise RuntimeError("no candidate policy fits this batch")
    ms, threads, ppt = min(results)
    px = sum(W * H for W, H in sizes)
    entry = {"threads": threads, "ppt": ppt, "solve_ms": round(ms, 4), "mpx_s_solve": round(px / ms / 1e3, 1),
             "candidates": {f"{t}x{p}": round(m, 4) for m, t, p in results}}
    key = cache_key(sizes, precision, n_gn, n_cg, _device_name())
    data = _load(path)
    data[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return entry


def tuned_policy(sizes: Sequence[Tuple[int, int]], precision: str = "bf16", n_gn: int = 10, n_cg: int = 20,
                 cache: Optional[str] = None, retune: bool = False) -> dict:
    """The cached policy for this size mix on this device, tuning it first if absent."""
    path = cache or os.environ.get("KF_TUNE_CACHE") or DEFAULT_CACHE
    key = cache_key(sizes, precision, n_gn, n_cg, _device_name())
    entry = None if retune else _load(path).get(key)
    if entry is None:
        entry = tune(sizes, precision, n_gn, n_cg, cache=path)
    return entry
