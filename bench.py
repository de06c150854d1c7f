"""Throughput / latency benchmark of the keyframe depth update on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --sync-sweep      (team-synchronisation latency vs team size)
    python bench.py --accuracy        (depth accuracy of the method's variants, synthetic scenes)

Workload (default): one 640 x 480 keyframe fused with a 30-frame sequence in the
precision form (bf16 keyframe image and patch buffers, fp32 maps and arithmetic,
fp64 CG dot products), N_s = 128 epipolar samples, 5 x 5 patch, 10 Gauss-Newton
iterations x 20 PCG iterations per frame. Inputs are seeded synthetic scenes,
resident in device memory before timing starts.

A step = keyframe init + 30 x (stereo update + solve) + depth read-out. The
steps run twice: on one stream (one frame in flight: per-frame fuse latency,
stage times, the solver launch's duration for the roofline figure) and with
frame pipelining (the next frame's stereo update overlaps the current solve on
a second stream; same results), which gives the headline Mpixel/s. Prints one
JSON line: Mpixel/s of fused frames (30 x 640 x 480 per step), p50/p99
per-frame fuse latency, the solver kernel's roofline figure, the CPU oracle
baseline and the precision form's error against it.

The same line carries, under "batched", the batched form: 64 keyframes of
mixed size (160x120, 320x240, 512x384, 640x480; bf16 images, f32 maps,
LINE5, N_s = 32, 10 x 20), each fused with one new frame per step by one
stereo and one persistent solver launch (graph replays).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused keyframe-update Mpixel/s at 640x480 + p50/p99 fuse latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solver_640x480_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solver_batched64_traffic.json")
SOLVER_SRCS = tuple(os.path.join(ROOT, "paper_2207_12244_amd", "csrc", f) for f in ("kf_solve.hip", "kf_internal.h"))

WORKLOAD = dict(config=2, W=640, H=480, frames=30, precision="bf16", pattern="sq5x5", n_samples=128,
                n_gn=10, n_cg=20)
BATCHED = dict(config=3, keyframes=64, precision="bf16", pattern="line5", n_samples=32, n_gn=10, n_cg=20)
SERVING = dict(config=4, streams=32, requests=40, keyframe_every=20, views=4, precision="f32", pattern="sq5x5",
               n_samples=64, n_gn=10, n_cg=20, budget_gib=64)


def solver_bytes_per_frame(N, n_gn, n_cg, word=4):
    """Algorithmic bytes of one frame's solve: per GN iteration assembly 13 words,
    PCG initialisation 7, each PCG iteration 9 (read x, r, p, diag, c_x, c_y;
    write x, r, p), scale step 3 -> (23 + 9 n_cg) words per pixel."""
    return n_gn * (23 + 9 * n_cg) * word * N


def source_hash(*paths):
    """sha256 (16 hex) of source files' code with comments and blank space
    removed, so that comment edits do not invalidate counters of an unchanged kernel."""
    import re
    text = ""
    for path in paths:
        with open(path) as f:
            t = f.read()
        t = re.sub(r"/\*.*?\*/", "", t, flags=re.S)
        t = re.sub(r"//[^\n]*", "", t)
        text += "\n".join(line.strip() for line in t.splitlines() if line.strip()) + "\n"
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def load_traffic(path=TRAFFIC_FILE, layout=None):
    """HBM bytes per solver launch from a committed rocprofv3 counter summary,
    or None when the solver source or the launch layout changed since the
    counters were taken."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("solver_source_sha256_16") != source_hash(*SOLVER_SRCS):
        return None
    if layout is not None and t.get("launch_layout") != layout:
        return None
    return t.get("hbm_bytes_per_launch")


def host_cpu():
    """Logical CPUs of the host and its CPU model (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cpus": os.cpu_count(), "cpu_model": model}


def oracle_pool(workers):
    """Processes for the oracle's per-pixel search (spawned: they never touch the GPU)."""
    import concurrent.futures
    import multiprocessing
    return concurrent.futures.ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("spawn"))


def gpu_states_per_frame(case, wl, torch):
    """The precision form run once more on one stream (untimed): log-depth x and
    the match indices after every frame, for the comparison with the oracle."""
    from paper_2207_12244_amd.kf import Keyframe
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    kf = Keyframe(case.W, case.H, precision=wl["precision"], pattern=wl["pattern"], n_samples=wl["n_samples"],
                  n_gn=wl["n_gn"], n_cg=wl["n_cg"], K=case.K)
    kf.set_prior(dev(case.image0, torch.uint8), *[dev(m, torch.float32) for m in case.priors.maps()], case.T_wc0)
    out = []
    for f in range(len(case.images)):
        kf.fuse_frame(dev(case.images[f], torch.uint8), case.poses[f])
        st = kf.export_state()
        out.append((st["x"].cpu().numpy().astype(np.float64), st["match"].cpu().numpy(), st["tau"]))
    kf.close()
    return out


def cpu_baseline_and_accuracy(case, wl, gpu_states, workers):
    """The FP64 oracle, as it stands, fused over the whole 30-frame sequence of
    one step (stereo over the textured pixels in row blocks on a process pool,
    10 x 20 Jacobi PCG fusion in this process), timed on the host; after every
    frame its depth is compared with the GPU form's."""
    from oracle import OracleKeyframe, SolverParams, StereoParams
    with oracle_pool(workers) as pool:
        ok = OracleKeyframe(case.K, case.W, case.H, StereoParams(n_samples=wl["n_samples"], pattern=wl["pattern"]),
                            SolverParams(n_gn=wl["n_gn"], n_cg=wl["n_cg"], linear_solver="pcg"), pool=pool,
                            n_blocks=2 * workers)
        ok.set_prior(case.image0, *case.priors.maps(), case.T_wc0)
        pool.submit(int, 0).result()   # workers up before the clock starts
        per_frame = []
        wall = 0.0
        for f in range(len(case.images)):
            w0 = time.perf_counter()
            rep = ok.fuse_frame(case.images[f], case.poses[f])
            wall += time.perf_counter() - w0
            x_g, match_g, tau_g = gpu_states[f]
            rel = np.abs(np.exp(x_g - ok.x) - 1.0)
            mism = int(np.count_nonzero(match_g.ravel()[rep.search.pix] != rep.search.k_best))
            per_frame.append({"frame": f + 1, "depth_rel_err_max": float(f"{rel.max():.4g}"),
                              "depth_rel_err_rms": float(f"{np.sqrt(np.mean(rel ** 2)):.4g}"),
                              "scale_rel_err": float(f"{abs(np.exp(tau_g - ok.tau) - 1.0):.4g}"),
                              "index_mismatch_rate": float(f"{mism / max(1, rep.search.pix.size):.4g}")})
            print(f"# oracle frame {f + 1}: {per_frame[-1]}", file=sys.stderr, flush=True)
    nF = len(case.images)
    base = {"value": round(nF * case.W * case.H / wall / 1e6, 6), "unit": "Mpixel/s", "cores": workers + 1,
            "kind": "oracle",
            "sample": f"the whole {nF}-frame sequence of one step ({case.W}x{case.H}, stereo on a {workers}-process "
                      f"pool, PCG fusion in the main process), {wall:.1f} s wall on the host",
            "seconds": round(wall, 3), **host_cpu()}
    last = per_frame[-1]
    acc = {"after_frame": nF, "depth_rel_err_max": last["depth_rel_err_max"],
           "depth_rel_err_rms": last["depth_rel_err_rms"], "scale_rel_err": last["scale_rel_err"],
           "worst_frame_rms": max(p["depth_rel_err_rms"] for p in per_frame),
           "worst_frame_index_mismatch_rate": max(p["index_mismatch_rate"] for p in per_frame),
           "against": "FP64 oracle run on its own over the same sequence, iteration-matched 10 x 20 Jacobi PCG; "
                      "the two drift apart through near-tie stereo decisions",
           "per_frame": per_frame}
    return base, acc


def _gen_batched_case(i):
    import kfsynth
    return kfsynth.config_case(BATCHED["config"], i)


def batched_cases(n):
    """The batched workload's keyframes (seeded size per keyframe), generated in a process pool."""
    import concurrent.futures
    import multiprocessing
    t_gen = time.perf_counter()
    workers = max(1, min(8, os.cpu_count() or 1))
    ctx = multiprocessing.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        cases = list(ex.map(_gen_batched_case, range(n)))
    print(f"# batched: generated {len(cases)} keyframes in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    return cases


def cpu_baseline_batched(cases, wl):
    """The FP64 oracle, as it stands, fusing one keyframe of each size in the
    batch with its frame (stereo + 10 x 20 PCG), timed on the host."""
    from oracle import OracleKeyframe, SolverParams, StereoParams
    picked = {}
    for c in cases:
        picked.setdefault((c.W, c.H), c)
    wall = cpu = 0.0
    px = 0
    for (W, H), case in sorted(picked.items()):
        ok = OracleKeyframe(case.K, W, H, StereoParams(n_samples=wl["n_samples"], pattern=wl["pattern"]),
                            SolverParams(n_gn=wl["n_gn"], n_cg=wl["n_cg"], linear_solver="pcg"))
        ok.set_prior(case.image0, *case.priors.maps(), case.T_wc0)
        w0, c0 = time.perf_counter(), time.process_time()
        ok.fuse_frame(case.images[0], case.poses[0])
        wall += time.perf_counter() - w0
        cpu += time.process_time() - c0
        px += W * H
    threads = max(1, int(round(cpu / wall)))
    sizes = ", ".join(f"{W}x{H}" for W, H in sorted(picked))
    return {"value": round(px / wall / 1e6, 6), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"one keyframe of each size in the batch ({sizes}) fused with its frame in one process "
                      f"(cores = CPU time / wall: numpy's threads), {wall:.1f} s wall",
            "seconds": round(wall, 3), **host_cpu()}


def run_batched(a, torch, cases):
    """Batched form: one step = one new frame fused into each of 64 keyframes."""
    from paper_2207_12244_amd.kf import Batch, Keyframe
    wl = BATCHED
    from paper_2207_12244_amd import autotune
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    t_tune = time.perf_counter()
    pol = autotune.tuned_policy([(c.W, c.H) for c in cases], wl["precision"], wl["n_gn"], wl["n_cg"])
    print(f"# batched: shape policy {pol['threads']} threads x {pol['ppt']} px/thread "
          f"({time.perf_counter() - t_tune:.1f}s)", file=sys.stderr, flush=True)
    members, imgs, poses = [], [], []
    for c in cases:
        kf = Keyframe(c.W, c.H, K=c.K, precision=wl["precision"], pattern=wl["pattern"], n_samples=wl["n_samples"],
                      n_gn=wl["n_gn"], n_cg=wl["n_cg"], solver_threads=pol["threads"],
                      tiles=autotune.tiles_for(c.W, c.H, pol["threads"], pol["ppt"]))
        kf.set_prior(dev(c.image0, torch.uint8), *[dev(m, torch.float32) for m in c.priors.maps()], c.T_wc0)
        members.append(kf)
        imgs.append(dev(c.images[0], torch.uint8))
        poses.append(c.poses[0])
    batch = Batch(members)
    stream = members[0].stream
    steps = a.batched_steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]

    def step(k):
        if k is not None:
            ev[k][0].record(stream)
        batch.stereo_update(imgs, poses)
        if k is not None:
            ev[k][1].record(stream)
        batch.solve()
        if k is not None:
            ev[k][2].record(stream)

    for _ in range(max(2, a.warmup)):
        step(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stereo_ms = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    solve_ms = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
    lat_ms = [ev[k][0].elapsed_time(ev[k][2]) for k in range(steps)]
    px = sum(c.W * c.H for c in cases)
    bpl = sum(solver_bytes_per_frame(c.W * c.H, wl["n_gn"], wl["n_cg"]) for c in cases)
    solve_avg_s = float(np.mean(solve_ms)) / 1000.0
    achieved = bpl / solve_avg_s / 1e9
    sizes = {}
    for c in cases:
        sizes[f"{c.W}x{c.H}"] = sizes.get(f"{c.W}x{c.H}", 0) + 1
    out = {
        "value": round(px * steps / total / 1e6, 3), "unit": "Mpixel/s", "steps": steps,
        "ms_per_step": round(1000.0 * total / steps, 3),
        "config": {"workload": f"{len(cases)} keyframes of mixed size, each fused with one new frame per step; "
                               f"bf16 images, f32 maps and arithmetic, LINE5, N_s={wl['n_samples']}, "
                               f"{wl['n_gn']} GN x {wl['n_cg']} PCG",
                   "sizes": sizes, "pixels_per_step": px,
                   "seeds": f"{kfsynth_seed(wl['config'], 0)}..{kfsynth_seed(wl['config'], len(cases) - 1)}",
                   "solver_launch": batch.layout(),
                   "shape_policy": {"threads": pol["threads"], "px_per_thread_cap": pol["ppt"]}},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "stage_ms_per_step": {"stereo": round(float(np.mean(stereo_ms)), 4),
                              "solve": round(float(np.mean(solve_ms)), 4)},
        "roofline": roofline_entry("k_solve_batch", bpl, solve_avg_s, load_traffic(BATCH_TRAFFIC_FILE, batch.layout())),
    }
    lay = batch.layout()
    out["roofline"]["dependent_syncs_longest_queue"] = lay["max_queue"] * members[0].stats().team_syncs
    batch.close()
    out["plain_same_workload"] = run_plain_batched(a, torch, cases, wl, imgs, poses, out["value"])
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(cases, wl)
    return out


def run_plain_batched(a, torch, cases, wl, imgs, poses, batched_value):
    """The plain form on the batched workload: one context per keyframe with the
    plain form's own (latency-optimal) tiling, a step = one kf_fuse_frame per
    keyframe on one stream. Results equal the batched form's bit for bit when
    the tilings match; here each keyframe keeps its own best tiling."""
    from paper_2207_12244_amd.kf import Keyframe
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    plain = []
    for c in cases:
        kf = Keyframe(c.W, c.H, K=c.K, precision=wl["precision"], pattern=wl["pattern"], n_samples=wl["n_samples"],
                      n_gn=wl["n_gn"], n_cg=wl["n_cg"])
        kf.set_prior(dev(c.image0, torch.uint8), *[dev(m, torch.float32) for m in c.priors.maps()], c.T_wc0)
        plain.append(kf)

    def pstep():
        for kf, im, po in zip(plain, imgs, poses):
            kf.fuse_frame(im, po)

    for _ in range(max(1, a.warmup)):
        pstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.batched_steps):
        pstep()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    for kf in plain:
        kf.close()
    px = sum(c.W * c.H for c in cases)
    value = px * a.batched_steps / total / 1e6
    return {"value": round(value, 3), "unit": "Mpixel/s", "ms_per_step": round(1000.0 * total / a.batched_steps, 3),
            "batched_speedup": round(batched_value / value, 3),
            "mode": f"{len(cases)} kf_fuse_frame calls per step on one stream, each keyframe with its own "
                    "latency-optimal tiling; same frames, poses and settings as the batched form"}


def roofline_entry(kernel, bpl, launch_s, traffic, sync=None):
    """The solver's roofline figures: algorithmic sweep bytes per launch / launch
    time against HBM peak (achieved, frac), the HBM bytes rocprofv3 counted per
    launch (traffic) and the rate they give, and the team-synchronisation floor.
    The vectors of a tile stay in registers and LDS, so the counted traffic is
    a small part of the sweeps: the launch is bound by the latency of its
    dependent team synchronisations, not by HBM."""
    achieved = bpl / launch_s / 1e9
    out = {"kernel": kernel, "bound": "latency", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "achieved_basis": "algorithmic sweep bytes (23 + 9 n_cg) x 4 B per pixel per GN iteration / launch time",
           "algorithmic_bytes_per_launch": bpl, "avg_launch_ms": round(launch_s * 1000.0, 4)}
    if traffic:
        out["counted_gbs"] = round(traffic / launch_s / 1e9, 2)
        out["counted_frac"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    if sync is not None:
        out["sync"] = sync
    return out


def kfsynth_seed(config, case):
    import kfsynth
    return kfsynth.seed_for(config, case)


def _gen_serving_stream(i):
    from kfsynth.serving import serving_stream
    w = SERVING
    return serving_stream(i, w["requests"], views=w["views"], keyframe_every=w["keyframe_every"])


def serving_streams(n):
    """The serving workload's request streams, generated in a process pool."""
    import concurrent.futures
    import multiprocessing
    t_gen = time.perf_counter()
    workers = max(1, min(8, os.cpu_count() or 1))
    ctx = multiprocessing.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        out = list(ex.map(_gen_serving_stream, range(n)))
    print(f"# serving: generated {len(out)} streams in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    return out


def run_serving(a, torch, streams):
    """Serving form: 32 camera streams with Poisson arrivals at 30 Hz each."""
    from paper_2207_12244_amd import autotune
    from paper_2207_12244_amd.serve import Request, Server
    w = SERVING
    sizes = [(c.W, c.H) for c, _ in streams]
    pol = autotune.tuned_policy(sizes, w["precision"], w["n_gn"], w["n_cg"]) if a.serving_tiles == "tuned" else None
    srv = Server(w["budget_gib"] << 30, precision=w["precision"], pattern=w["pattern"], n_samples=w["n_samples"],
                 n_gn=w["n_gn"], n_cg=w["n_cg"], solver_threads=pol["threads"] if pol else 512,
                 px_per_thread=pol["ppt"] if pol else None)
    for c, _ in streams:
        srv.open_stream(c.W, c.H, c.K)
    srv.start()

    def submit_all(offset):
        for sid, (c, reqs) in enumerate(streams):
            for r in reqs:
                srv.submit(sid, Request(r["kind"], r["t"] + offset, r["image"], r["pose"], r.get("priors")))

    # warm-up pass over the same requests (graphs, clocks), then the measured pass
    submit_all(0.0)
    srv.run()
    submit_all(0.0)
    st = srv.run()
    # capacity: the same requests arriving 20x faster (600 Hz per stream), far beyond what the device sustains
    for sid, (c, reqs) in enumerate(streams):
        for r in reqs:
            srv.submit(sid, Request(r["kind"], r["t"] / 20.0, r["image"], r["pose"], r.get("priors")))
    cap = srv.run()
    hist = {}
    for W, H in sizes:
        hist[f"{W}x{H}"] = hist.get(f"{W}x{H}", 0) + 1
    out = {"value": round(st["mpx_s"], 3), "unit": "Mpixel/s",
           "latency_ms": {k: round(v, 4) for k, v in st["latency_ms"].items()},
           "frames": st["frames"], "seconds": round(st["seconds"], 3), "calls": st["calls"],
           "mean_streams_per_call": round(st["mean_streams_per_call"], 2),
           "capacity": {"mpx_s": round(cap["mpx_s"], 3), "arrivals": "same requests at 20x the rate",
                        "latency_ms": {k: round(v, 4) for k, v in cap["latency_ms"].items()},
                        "mean_streams_per_call": round(cap["mean_streams_per_call"], 2)},
           "config": {"workload": f"{len(streams)} camera streams, Poisson arrivals at 30 Hz each, a new keyframe "
                                  f"every {w['keyframe_every']} requests, f32 maps, SQ5X5, N_s={w['n_samples']}, "
                                  f"{w['n_gn']} GN x {w['n_cg']} PCG; latency = completion - arrival incl. the "
                                  "host-to-device copy of the frame",
                      "sizes": hist, "requests_per_stream": w["requests"],
                      "hbm_budget_bytes": srv.budget, "hbm_admitted_bytes": srv.used,
                      "shape_policy": {"threads": pol["threads"], "px_per_thread_cap": pol["ppt"]} if pol
                      else "latency-optimal per size"}}
    srv.close()
    out["plain_capacity"] = run_plain_serving(torch, streams, w, out["capacity"]["mpx_s"])
    return out


def run_plain_serving(torch, streams, w, served_capacity):
    """The plain form on the serving requests at full rate: one context per
    stream, every request in arrival order as one kf_set_prior / kf_fuse_frame
    call on one stream, inputs already on the device."""
    from paper_2207_12244_amd.kf import Keyframe
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    kfs = [Keyframe(c.W, c.H, K=c.K, precision=w["precision"], pattern=w["pattern"], n_samples=w["n_samples"],
                    n_gn=w["n_gn"], n_cg=w["n_cg"]) for c, _ in streams]
    cache = {}

    def up(arr, dt):
        key = id(arr)
        if key not in cache:
            cache[key] = (arr, dev(arr, dt))
        return cache[key][1]

    reqs = sorted(((r["t"], sid, i) for sid, (_, rs) in enumerate(streams) for i, r in enumerate(rs)))
    calls = []
    for _, sid, i in reqs:
        r = streams[sid][1][i]
        if r["kind"] == "keyframe":
            calls.append((sid, up(r["image"], torch.uint8), [up(m, torch.float32) for m in r["priors"]], r["pose"]))
        else:
            calls.append((sid, up(r["image"], torch.uint8), None, r["pose"]))

    def run():
        px = 0
        for sid, img, pri, pose in calls:
            if pri is not None:
                kfs[sid].set_prior(img, *pri, pose)
            else:
                kfs[sid].fuse_frame(img, pose)
                px += kfs[sid].W * kfs[sid].H
        return px

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    px = run()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    for kf in kfs:
        kf.close()
    value = px / total / 1e6
    return {"mpx_s": round(value, 3), "served_capacity_speedup": round(served_capacity / value, 3),
            "mode": "every request of the serving workload in arrival order as one plain call on one stream, "
                    "inputs resident (the served figure includes its host-to-device copies)"}


def run_headline(a, torch):
    """The headline workload: one 640 x 480 keyframe fused with a 30-frame sequence."""
    import kfsynth
    from paper_2207_12244_amd.kf import Keyframe
    wl = WORKLOAD
    t_gen = time.perf_counter()
    case = kfsynth.config_case(wl["config"], 0)
    print(f"# generated {case.W}x{case.H} keyframe + {len(case.images)} frames in "
          f"{time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    img0 = dev(case.image0, torch.uint8)
    priors = [dev(m, torch.float32) for m in case.priors.maps()]
    frames = [dev(im, torch.uint8) for im in case.images]
    poses = case.poses
    tiles = tuple(int(v) for v in a.tiles.lower().split("x"))
    nF = len(frames)

    def timed(pipe):
        """Timed steps of one context; with pipe the next frame's stereo overlaps
        the current solve (pipeline_frames). Returns the context, total seconds
        and per-frame stereo / solve / latency lists (HIP events)."""
        kf = Keyframe(case.W, case.H, precision=wl["precision"], pattern=wl["pattern"], n_samples=wl["n_samples"],
                      n_gn=wl["n_gn"], n_cg=wl["n_cg"], K=case.K, tiles=tiles, solver_threads=a.solver_threads,
                      cooperative=a.cooperative, cg_variant=a.cg_variant, pipeline_frames=pipe)
        us, ss = kf.stream, kf.solve_stream()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(nF)]

        def step(record):
            kf.set_prior(img0, *priors, case.T_wc0)
            for f in range(nF):
                if record:
                    ev[f][0].record(us)
                kf.stereo_update(frames[f], poses[f])
                if record:
                    ev[f][1].record(us)
                kf.solve()
                if record:
                    ev[f][2].record(ss)
            return kf.read_depth()

        for _ in range(a.warmup):
            step(False)
        torch.cuda.synchronize()
        stereo, solve, lat = [], [], []
        total = 0.0
        for _ in range(a.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(True)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            for f in range(nF):
                stereo.append(ev[f][0].elapsed_time(ev[f][1]))
                solve.append(ev[f][1].elapsed_time(ev[f][2]))
                lat.append(ev[f][0].elapsed_time(ev[f][2]))
        return kf, total, stereo, solve, lat

    # one stream (one frame in flight): per-frame latency, stage times and the
    # solver's launch duration; then the pipelined context for the throughput
    kf, total1, stereo_ms, solve_ms, lat_ms = timed(False)
    solver_layout = kf.solver_layout()
    syncs = kf.stats().team_syncs
    sync = sync_floor(kf, torch, syncs, float(np.mean(solve_ms)))
    kf.close()
    kf, total, _, _, lat_p = timed(True)
    st = kf.stats()
    kf.close()
    ms_per_step = 1000.0 * total / a.steps
    px = nF * case.W * case.H
    value = px / (ms_per_step / 1000.0) / 1e6
    N = case.W * case.H
    bpl = solver_bytes_per_frame(N, wl["n_gn"], wl["n_cg"])
    solve_avg_s = float(np.mean(solve_ms)) / 1000.0
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{case.W}x{case.H} keyframe + {nF}-frame sequence, precision form (keyframe image stored "
                        f"as bf16, which is exact for uint8 images: with the 5x5 patch at integer keyframe pixels "
                        f"no value is rounded to bf16, so the form computes as F32; f32 maps and arithmetic; CG inner "
                        f"products accumulated in f64 and exchanged between workgroups with a 2^-37 relative "
                        f"rounding), N_s={wl['n_samples']}, 5x5 patch, {wl['n_gn']} GN x {wl['n_cg']} PCG per frame",
            "frames_per_step": nF, "width": case.W, "height": case.H, "seed": kfsynth.seed_for(wl["config"], 0),
            "solver_layout": solver_layout, "pipeline_frames": 1,
            "solver_launch": "cooperative" if a.cooperative else "plain",
            "cg_variant": "pipelined" if a.cg_variant in ("auto", "pipelined") else "textbook",
        },
        "latency_ms": {"p50": round(float(np.percentile(lat_p, 50)), 4),
                       "p99": round(float(np.percentile(lat_p, 99)), 4),
                       "mode": "measured with the value (pipeline_frames=1, frames back to back): stereo start to "
                               "solve end; a frame waits for the previous frame's solve"},
        "single_stream": {"value": round(px / (total1 / a.steps) / 1e6, 3),
                          "ms_per_step": round(1000.0 * total1 / a.steps, 3),
                          "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                                         "p99": round(float(np.percentile(lat_ms, 99)), 4),
                                         "mode": "one frame in flight: stereo start to solve end"}},
        "stage_ms_per_frame": {"stereo": round(float(np.mean(stereo_ms)), 4),
                               "solve": round(float(np.mean(solve_ms)), 4)},
        "frame_stats": {"textured": st.n_searched, "semi_valid": st.n_valid, "scale": round(st.scale, 6),
                        "team_syncs_per_solve": syncs},
        "roofline": roofline_entry("k_solve", bpl, solve_avg_s, load_traffic(TRAFFIC_FILE, solver_layout), sync),
        "context": {"paper": "16 ms semi-dense + 33 ms optimisation per frame on i7-5820K + GTX 980, "
                             "resolution unstated (Table IV)"},
    }
    if not a.no_cpu_baseline:
        gpu_states = gpu_states_per_frame(case, wl, torch)
        workers = max(1, min(8, os.cpu_count() or 1))
        out["cpu_baseline"], out["accuracy"] = cpu_baseline_and_accuracy(case, wl, gpu_states, workers)
    return out


def probe_us_per_sync(kf, torch, rounds, nvalues=2, repeats=3):
    """Microseconds per round of the synchronisation probe (kf_probe_sync), one
    warm-up launch, then the fastest of `repeats` launches timed with HIP events
    on the context's stream."""
    kf.probe_sync(rounds, nvalues)
    best = None
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(kf.stream)
        kf.probe_sync(rounds, nvalues)
        e1.record(kf.stream)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1000.0 / rounds
        best = us if best is None else min(best, us)
    return best


def sync_floor(kf, torch, syncs, solve_ms, rounds=2000):
    """Team-synchronisation floor of the solve: the probe launch (same team,
    tiling and exchange as the solve, no arithmetic) timed with HIP events on
    the context's stream; floor = synchronisations per solve x time per probe
    round."""
    best = probe_us_per_sync(kf, torch, rounds)
    floor_ms = syncs * best / 1000.0
    return {"syncs_per_launch": syncs, "probe_us_per_sync": round(best, 4), "floor_ms": round(floor_ms, 4),
            "frac": round(floor_ms / solve_ms, 4),
            "probe": f"kf_probe_sync: {rounds} exchanges of 2 partials + the tile boundary, same team and tiling "
                     "as the solve, no arithmetic; fastest of 3 launches"}


# team shapes (tiles_x, tiles_y) of the synchronisation sweep, up to the largest
# team of one keyframe (256 workgroups); every tile is 40 x 30 pixels, the
# 640 x 480 solve's tile at 16 x 16
SYNC_SWEEP_TEAMS = ((1, 1), (2, 1), (2, 2), (4, 4), (8, 4), (8, 8), (10, 10), (12, 12), (16, 12), (16, 16))
SYNC_SWEEP_TILE = (40, 30)


def run_sync_sweep(torch, rounds=2000, threads=512):
    """Exchange latency against team size: for each team shape a keyframe of
    (40 tiles_x) x (30 tiles_y) pixels at that tiling, and the probe's time per
    synchronisation with 1, 2 and 3 published values (a CG iteration of the
    pipelined solve publishes 2, the textbook one 1 per synchronisation), in the
    float forms (one 64-bit word per partial) and FP64 (two words)."""
    from paper_2207_12244_amd.kf import Keyframe, KfError
    rows = []
    for precision in ("f32", "f64"):
        for tx, ty in SYNC_SWEEP_TEAMS:
            W, H = SYNC_SWEEP_TILE[0] * tx, SYNC_SWEEP_TILE[1] * ty
            row = {"precision": precision, "tiles": [tx, ty], "workgroups": tx * ty, "size": [W, H],
                   "threads": threads}
            try:
                kf = Keyframe(W, H, precision=precision, pattern="sq5x5", n_samples=128, tiles=(tx, ty),
                              solver_threads=threads)
            except KfError as e:
                rows.append({**row, "skipped": str(e)})
                continue
            dt = kf.dtype
            zero = torch.zeros((H, W), dtype=dt, device="cuda")
            one = torch.ones((H, W), dtype=dt, device="cuda")
            img = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
            kf.set_prior(img, zero, one, zero, one, zero, one, np.eye(4))
            try:
                row["us_per_sync"] = {str(nv): round(probe_us_per_sync(kf, torch, rounds, nv), 4) for nv in (1, 2, 3)}
            except KfError as e:
                row["skipped"] = str(e)
            kf.close()
            rows.append(row)
            print(f"# sync sweep {precision} {tx}x{ty} ({tx * ty} workgroups, {W}x{H}): "
                  f"{row.get('us_per_sync', row.get('skipped'))}", file=sys.stderr, flush=True)
    return {"sync_sweep": rows, "rounds": rounds,
            "probe": "kf_probe_sync: per round, every workgroup publishes nvalues partials and its tile boundary "
                     "and polls the team's partials and its neighbours' boundaries, no arithmetic; us per round = "
                     "the fastest of 3 launches timed with HIP events, after one warm-up launch"}


# accuracy of the method's variants on the synthetic headline scenes: the
# share of depth values within 10 % of the ground truth (Sec. III's measure)
ACCURACY_CASES = (0, 1, 2)
ACCURACY_VARIANTS = (
    ("network prior only", None),
    ("full cost, Huber", {}),
    ("full cost, Tukey (c = 4.685)", dict(robust="tukey", huber_delta=4.685)),
    ("no pairwise terms (Table III)", dict(variant="no_pairwise")),
    ("least-squares scale post-fit (Table II)", dict(variant="scale_postfit")),
)


def run_accuracy(torch):
    """Each variant fuses the 30-frame 640 x 480 headline sequence (precision
    form, SQ5X5, N_s = 128, 10 x 20) of three seeded synthetic scenes; the
    fused depth is compared with the rendered ground truth of the keyframe.
    "network prior only" reads the depth right after the keyframe is set."""
    import kfsynth
    from paper_2207_12244_amd.kf import Keyframe
    wl = WORKLOAD
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    per = {name: [] for name, _ in ACCURACY_VARIANTS}
    for c in ACCURACY_CASES:
        case = kfsynth.config_case(wl["config"], c)
        gt = case.depth0.astype(np.float64)
        img0 = dev(case.image0, torch.uint8)
        priors = [dev(m, torch.float32) for m in case.priors.maps()]
        frames = [dev(im, torch.uint8) for im in case.images]
        for name, kw in ACCURACY_VARIANTS:
            kf = Keyframe(case.W, case.H, precision=wl["precision"], pattern=wl["pattern"], n_samples=wl["n_samples"],
                          n_gn=wl["n_gn"], n_cg=wl["n_cg"], K=case.K, **(kw or {}))
            kf.set_prior(img0, *priors, case.T_wc0)
            if kw is not None:
                for f, im in enumerate(frames):
                    kf.fuse_frame(im, case.poses[f])
            d, _ = kf.read_depth()
            kf.close()
            rel = np.abs(d.cpu().numpy().astype(np.float64) - gt) / gt
            per[name].append({"case": c, "pct_within_10": round(100.0 * float(np.mean(rel < 0.1)), 2),
                              "mean_abs_rel": round(float(np.mean(rel)), 4)})
            print(f"# accuracy case {c} {name}: {per[name][-1]}", file=sys.stderr, flush=True)
    out = {}
    for name, rows in per.items():
        out[name] = {"pct_within_10": round(float(np.mean([r["pct_within_10"] for r in rows])), 2),
                     "mean_abs_rel": round(float(np.mean([r["mean_abs_rel"] for r in rows])), 4), "per_case": rows}
    return {"accuracy_synthetic": out,
            "workload": f"{len(ACCURACY_CASES)} seeded synthetic 640x480 scenes (config 2 cases "
                        f"{list(ACCURACY_CASES)}), 30 frames each, {wl['precision']} form, {wl['pattern']}, "
                        f"N_s={wl['n_samples']}, {wl['n_gn']} GN x {wl['n_cg']} PCG; ground truth = rendered "
                        "keyframe depth; measure = share of pixels with |d - d_gt| / d_gt < 0.1"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiles", default="0x0", help="solver tile grid TXxTY (0x0 = automatic)")
    ap.add_argument("--solver-threads", type=int, default=0, help="solver workgroup size (0 = automatic)")
    ap.add_argument("--cooperative", action="store_true", help="launch the solver cooperatively")
    ap.add_argument("--cg-variant", default="auto", choices=["auto", "textbook", "pipelined"])
    ap.add_argument("--form", default="all", choices=["all", "headline", "batched", "serving"],
                    help="headline 640x480 sequence, the batched or serving form, or all three "
                         "(batched and serving under their own keys)")
    ap.add_argument("--serving-tiles", default="auto", choices=["tuned", "auto"],
                    help="serving tile shapes: latency-optimal per size (auto) or the batch autotuner's")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--accuracy", action="store_true",
                    help="only the depth accuracy of the method's variants on synthetic scenes")
    ap.add_argument("--sync-sweep", action="store_true",
                    help="only measure the team-synchronisation latency against team size (kf_probe_sync)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device-to-device copy (HBM counter calibration)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); "
              "independent keyframes shard across GPUs without communication, see the design notes.",
              file=sys.stderr)
        return 2

    if a.accuracy:
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 2
        print(json.dumps(run_accuracy(torch)), flush=True)
        return 0
    if a.sync_sweep:
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 2
        print(json.dumps(run_sync_sweep(torch)), flush=True)
        return 0

    # the batched and serving workloads are generated in process pools before the GPU is touched
    batched_in = batched_cases(BATCHED["keyframes"]) if a.form in ("all", "batched") else None
    serving_in = serving_streams(SERVING["streams"]) if a.form in ("all", "serving") else None

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if a.calibrate_copy:
        # known traffic: reads 256 MiB and writes 256 MiB
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.form == "batched":
        out = run_batched(a, torch, batched_in)
        out = {"metric": "batched keyframe-update Mpixel/s (64 mixed-size keyframes)", **out, "n_gpus": 1,
               "warmup": a.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic"}
    elif a.form == "serving":
        out = run_serving(a, torch, serving_in)
        out = {"metric": "served keyframe-update Mpixel/s + p50/p99 latency (32 streams)", **out, "n_gpus": 1,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    else:
        out = run_headline(a, torch)
        if batched_in is not None:
            out["batched"] = run_batched(a, torch, batched_in)
        if serving_in is not None:
            out["serving"] = run_serving(a, torch, serving_in)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
