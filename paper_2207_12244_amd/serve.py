"""Serving loop: many camera streams, each with a resident keyframe, fused
continuously as their frames arrive.

Every admitted stream owns one keyframe context (its resident state and
solver scratch), two device frame slots and pinned host staging. Frames
arrive on the host at their own times; the loop copies each arrived frame to
its stream's free slot on a copy stream and, whenever the compute stream is
free to take more work, fuses at most one ready frame per stream in one
batched call (kf_batch_fuse_subset) on the compute stream. A stream's frames
stay in order: a stream with a frame in flight joins no further call until
that frame is done. Latency is completion minus arrival, both on the host
clock; completion is observed by polling the call's event.

Admission is by device-memory budget: a stream is admitted only if its
resident and in-flight bytes fit in what the budget has left.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from .kf import Batch, Keyframe, kf_workspace_bytes


class AdmissionError(RuntimeError):
    """A stream does not fit in the remaining device-memory budget."""


@dataclass
class _Stream:
    sid: int
    W: int
    H: int
    kf: Keyframe
    slots: list                      # two device frame buffers
    pinned: list                     # two pinned host staging buffers
    slot_free: list                  # slot not referenced by a queued or running call
    copy_done: list                  # event per slot: its upload finished
    prior_dev: list                  # device staging of a new keyframe's priors
    prior_done: object               # event: the staged priors are on the device
    queue: collections.deque = field(default_factory=collections.deque)
    inflight: bool = False
    next_slot: int = 0


@dataclass
class Request:
    """One item of a stream's input, in arrival order. kind "keyframe": a new
    keyframe (image0 + six prior maps + pose) replaces the stream's state;
    kind "frame": a new frame (image + pose) to fuse."""
    kind: str
    t_arrival: float
    image: np.ndarray
    pose: np.ndarray
    priors: Optional[Sequence[np.ndarray]] = None


class Server:
    def __init__(self, hbm_budget_bytes: int, *, precision: str = "f32", pattern: str = "sq5x5",
                 n_samples: int = 64, n_gn: int = 10, n_cg: int = 20, solver_threads: int = 512,
                 px_per_thread: Optional[int] = None):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.used = 0
        self.kw = dict(precision=precision, pattern=pattern, n_samples=n_samples, n_gn=n_gn, n_cg=n_cg)
        self.threads = solver_threads
        self.ppt = px_per_thread
        self.compute = torch.cuda.Stream()
        self.copy = torch.cuda.Stream()
        self.streams: List[_Stream] = []
        self.batch: Optional[Batch] = None
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.elt = 8 if precision == "f64" else 4

    # ------------------------------------------------------------ admission

    def _tiles(self, W, H):
        if self.ppt is None:
            return (0, 0)
        from .autotune import tiles_for
        return tiles_for(W, H, self.threads, self.ppt)

    def stream_bytes(self, W: int, H: int) -> int:
        """Device bytes one stream holds: the context workspace (resident state
        and solver scratch), two frame slots and the prior staging (image + 6 maps)."""
        from .kf import kf_config_default, KfError, PRECISIONS, PATTERNS
        cfg = kf_config_default(W, H)
        cfg.precision = PRECISIONS[self.kw["precision"]]
        cfg.pattern = PATTERNS[self.kw["pattern"]]
        cfg.n_samples, cfg.n_gn, cfg.n_cg = self.kw["n_samples"], self.kw["n_gn"], self.kw["n_cg"]
        cfg.solver_threads = self.threads
        cfg.solver_tiles_x, cfg.solver_tiles_y = self._tiles(W, H)
        ws = kf_workspace_bytes(cfg)
        if ws == 0:
            raise KfError(-1, f"no valid configuration for {W}x{H}")
        return ws + 256 + 2 * W * H + W * H + 6 * W * H * self.elt

    def open_stream(self, W: int, H: int, K) -> int:
        if self.batch is not None:
            raise RuntimeError("streams are admitted before start()")
        need = self.stream_bytes(W, H)
        if self.used + need > self.budget:
            raise AdmissionError(f"stream {W}x{H} needs {need} B; {self.budget - self.used} B of the budget left")
        torch = self.torch
        kf = Keyframe(W, H, K=K, tiles=self._tiles(W, H), solver_threads=self.threads, stream=self.compute,
                      **self.kw)
        slots = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)]
        pinned = [torch.empty((H, W), dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        prior_dev = [torch.empty((H, W), dtype=torch.uint8, device="cuda")] + \
                    [torch.empty((H, W), dtype=self.dtype, device="cuda") for _ in range(6)]
        s = _Stream(len(self.streams), W, H, kf, slots, pinned, [True, True],
                    [torch.cuda.Event() for _ in range(2)], prior_dev, torch.cuda.Event())
        self.streams.append(s)
        self.used += need
        return s.sid

    def start(self):
        """Binds the admitted streams into one batch (its small table workspace
        is counted against the budget too)."""
        if not self.streams:
            raise RuntimeError("no stream admitted")
        self.batch = Batch([s.kf for s in self.streams])
        self.used += int(self.batch.workspace.numel())
        if self.used > self.budget:
            raise AdmissionError("the batch tables do not fit in the budget")

    # ------------------------------------------------------------ requests

    def submit(self, sid: int, req: Request):
        """Queues a request (host arrays); prior maps are converted to the map
        element type here, outside the serving loop."""
        if req.priors is not None:
            npdt = np.float64 if self.elt == 8 else np.float32
            req.priors = [np.ascontiguousarray(m, dtype=npdt) for m in req.priors]
        self.streams[sid].queue.append(req)

    def _upload(self, s: _Stream, req: Request, slot: int):
        """Copies a frame (or a keyframe's image and priors) to the device on the copy stream."""
        torch = self.torch
        with torch.cuda.stream(self.copy):
            if req.kind == "keyframe":
                s.prior_dev[0].copy_(torch.from_numpy(np.ascontiguousarray(req.image)))
                for dst, m in zip(s.prior_dev[1:], req.priors):
                    dst.copy_(torch.from_numpy(m))
                s.prior_done.record(self.copy)
            else:
                s.pinned[slot].numpy()[...] = req.image
                s.slots[slot].copy_(s.pinned[slot], non_blocking=True)
                s.copy_done[slot].record(self.copy)

    # ------------------------------------------------------------ loop

    def run(self, clock_start: Optional[float] = None, poll_sleep: float = 2e-5, max_calls_in_flight: int = 2) -> Dict:
        """Serves every submitted request in real time (arrival times are seconds
        after clock_start) and returns per-frame latencies and throughput.

        At most `max_calls_in_flight` batched calls are queued on the device at a
        time (one running, one waiting); frames that become ready meanwhile wait
        on the host and join the next call, so calls grow with the load."""
        torch = self.torch
        t0 = time.perf_counter() if clock_start is None else clock_start
        inflight = collections.deque()        # (event, [(stream, slot, req)])
        uploaded = {s.sid: collections.deque() for s in self.streams}   # (slot, req) copied or copying
        lat, px_done, n_calls, sizes = [], 0, 0, []
        remaining = sum(len(s.queue) for s in self.streams)
        t_first = min((s.queue[0].t_arrival for s in self.streams if s.queue), default=0.0)
        while remaining:
            now = time.perf_counter() - t0
            # uploads of arrived requests into free slots
            for s in self.streams:
                while s.queue and s.queue[0].t_arrival <= now:
                    req = s.queue[0]
                    if req.kind == "keyframe":
                        if s.inflight or uploaded[s.sid]:
                            break          # the new keyframe replaces the state: wait for earlier frames
                        s.queue.popleft()
                        self._upload(s, req, 0)
                        with torch.cuda.stream(self.compute):
                            self.compute.wait_event(s.prior_done)
                            s.kf.set_prior(*s.prior_dev, req.pose)
                        remaining -= 1
                        continue
                    slot = s.next_slot
                    if not s.slot_free[slot]:
                        break
                    s.queue.popleft()
                    s.slot_free[slot] = False
                    s.next_slot ^= 1
                    self._upload(s, req, slot)
                    uploaded[s.sid].append((slot, req))
            # one call with at most one ready frame per stream
            active, imgs, poses, items = [], [], [], []
            for s in self.streams:
                if len(inflight) >= max_calls_in_flight:
                    break
                if s.inflight or not uploaded[s.sid]:
                    continue
                slot, req = uploaded[s.sid].popleft()
                self.compute.wait_event(s.copy_done[slot])
                active.append(s.sid)
                imgs.append(s.slots[slot])
                poses.append(req.pose)
                items.append((s, slot, req))
                s.inflight = True
            if active:
                with torch.cuda.stream(self.compute):
                    self.batch.fuse_subset(active, imgs, poses)
                    ev = torch.cuda.Event()
                    ev.record(self.compute)
                inflight.append((ev, items))
                n_calls += 1
                sizes.append(len(active))
            # completions
            while inflight and inflight[0][0].query():
                _, items = inflight.popleft()
                t_done = time.perf_counter() - t0
                for s, slot, req in items:
                    lat.append(t_done - req.t_arrival)
                    px_done += s.W * s.H
                    s.inflight = False
                    s.slot_free[slot] = True
                    remaining -= 1
            if not active and poll_sleep:
                time.sleep(poll_sleep)
        torch.cuda.synchronize()
        span = time.perf_counter() - t0 - t_first     # first arrival to last completion
        lat_ms = np.asarray(lat) * 1000.0
        return {"frames": len(lat), "pixels": px_done, "seconds": span,
                "mpx_s": px_done / span / 1e6 if span > 0 else 0.0,
                "latency_ms": {"p50": float(np.percentile(lat_ms, 50)) if len(lat) else None,
                               "p99": float(np.percentile(lat_ms, 99)) if len(lat) else None,
                               "max": float(lat_ms.max()) if len(lat) else None},
                "calls": n_calls, "mean_streams_per_call": float(np.mean(sizes)) if sizes else 0.0}

    def close(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        for s in self.streams:
            s.kf.close()
