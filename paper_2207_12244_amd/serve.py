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
resident and in-flight bytes fit in what the budget has left. Streams can be
requested while the loop runs: a request waits (its frames queue up) until
enough memory is free, e.g. after an earlier stream has finished and closed;
the batch is then rebuilt over the new set of streams between two calls.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence

import numpy as np

from .kf import Batch, Keyframe, kf_workspace_bytes


class AdmissionError(RuntimeError):
    """A stream does not fit in the (remaining) device-memory budget."""


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


@dataclass
class _Stream:
    sid: int
    W: int
    H: int
    K: np.ndarray
    need: int                        # admitted device bytes
    close_when_done: bool = False
    queue: collections.deque = field(default_factory=collections.deque)
    kf: Optional[Keyframe] = None
    slots: list = field(default_factory=list)        # two device frame buffers
    pinned: list = field(default_factory=list)       # two pinned host staging buffers
    slot_free: list = field(default_factory=lambda: [True, True])
    copy_done: list = field(default_factory=list)    # event per slot: its upload finished
    prior_dev: list = field(default_factory=list)    # device staging of a new keyframe's priors
    prior_done: object = None                        # event: the staged priors are on the device
    uploaded: collections.deque = field(default_factory=collections.deque)   # (slot, request)
    inflight: bool = False
    next_slot: int = 0


class Server:
    def __init__(self, hbm_budget_bytes: int, *, precision: str = "f32", pattern: str = "sq5x5",
                 n_samples: int = 64, n_gn: int = 10, n_cg: int = 20, solver_threads: int = 512,
                 px_per_thread: Optional[int] = None, keep_results: bool = False):
        import torch
        self.keep_results = keep_results
        self.results = {}                              # sid -> final state of a closed stream (keep_results)
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.used = 0
        self.kw = dict(precision=precision, pattern=pattern, n_samples=n_samples, n_gn=n_gn, n_cg=n_cg)
        self.threads = solver_threads
        self.ppt = px_per_thread
        self.compute = torch.cuda.Stream()
        self.copy = torch.cuda.Stream()
        self.streams: Dict[int, _Stream] = {}          # admitted
        self.waiting: collections.deque = collections.deque()   # requested, not yet admitted
        self.batch: Optional[Batch] = None
        self.batch_bytes = 0
        self.member: Dict[int, int] = {}               # sid -> index in the batch
        self.dirty = False
        self.next_sid = 0
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.elt = 8 if precision == "f64" else 4
        self.admissions = []                           # (sid, time) of streams admitted while running
        self.closes = []                               # (sid, time) of streams closed while running

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

    def _materialise(self, s: _Stream):
        torch = self.torch
        W, H = s.W, s.H
        s.kf = Keyframe(W, H, K=s.K, tiles=self._tiles(W, H), solver_threads=self.threads, stream=self.compute,
                        **self.kw)
        s.slots = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)]
        s.pinned = [torch.empty((H, W), dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        s.prior_dev = [torch.empty((H, W), dtype=torch.uint8, device="cuda")] + \
                      [torch.empty((H, W), dtype=self.dtype, device="cuda") for _ in range(6)]
        s.copy_done = [torch.cuda.Event() for _ in range(2)]
        s.prior_done = torch.cuda.Event()
        self.streams[s.sid] = s
        self.used += s.need
        self.dirty = True

    def open_stream(self, W: int, H: int, K) -> int:
        """Admits a stream now, or raises AdmissionError."""
        need = self.stream_bytes(W, H)
        if self.used + need > self.budget:
            raise AdmissionError(f"stream {W}x{H} needs {need} B; {self.budget - self.used} B of the budget left")
        s = _Stream(self.next_sid, W, H, np.asarray(K, dtype=np.float64), need)
        self.next_sid += 1
        self._materialise(s)
        return s.sid

    def request_stream(self, W: int, H: int, K, requests: Sequence[Request], close_when_done: bool = True) -> int:
        """Queues a stream for admission once its first request has arrived and
        memory allows (streams are admitted in request order); its requests are
        served in order after that, and with close_when_done its memory is
        released after the last one. Raises AdmissionError if it could never
        fit in the budget."""
        need = self.stream_bytes(W, H)
        if need > self.budget:
            raise AdmissionError(f"stream {W}x{H} needs {need} B, more than the whole budget ({self.budget} B)")
        s = _Stream(self.next_sid, W, H, np.asarray(K, dtype=np.float64), need, close_when_done)
        self.next_sid += 1
        for r in requests:
            self._convert(r)
            s.queue.append(r)
        self.waiting.append(s)
        return s.sid

    def _close_stream(self, s: _Stream):
        if self.keep_results:
            self.results[s.sid] = s.kf.export_state()     # synchronises the compute stream
        s.kf.close()
        s.kf = None
        s.slots, s.pinned, s.prior_dev = [], [], []
        del self.streams[s.sid]
        self.used -= s.need
        self.dirty = True

    def _rebuild(self):
        """New batch over the admitted streams (no call may be in flight)."""
        if self.batch is not None:
            self.batch.close()
            self.used -= self.batch_bytes
            self.batch, self.batch_bytes = None, 0
        sids = sorted(self.streams)
        self.member = {sid: i for i, sid in enumerate(sids)}
        if sids:
            self.batch = Batch([self.streams[sid].kf for sid in sids])
            self.batch_bytes = int(self.batch.workspace.numel())
            self.used += self.batch_bytes
        self.dirty = False

    def start(self):
        """Binds the admitted streams into one batch (its small table workspace
        is counted against the budget too)."""
        if not self.streams:
            raise RuntimeError("no stream admitted")
        self._rebuild()
        if self.used > self.budget:
            raise AdmissionError("the batch tables do not fit in the budget")

    # ------------------------------------------------------------ requests

    def _convert(self, req: Request):
        """Prior maps to the map element type (done when queued, outside the loop)."""
        if req.priors is not None:
            npdt = np.float64 if self.elt == 8 else np.float32
            req.priors = [np.ascontiguousarray(m, dtype=npdt) for m in req.priors]

    def submit(self, sid: int, req: Request):
        """Queues a request (host arrays) of an admitted stream."""
        self._convert(req)
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
        """Serves the requests of every admitted and requested stream in real
        time (arrival times are seconds after clock_start) and returns
        per-frame latencies and throughput.

        At most `max_calls_in_flight` batched calls are queued on the device at a
        time (one running, one waiting); frames that become ready meanwhile wait
        on the host and join the next call, so calls grow with the load."""
        torch = self.torch
        t0 = time.perf_counter() if clock_start is None else clock_start
        inflight = collections.deque()        # (event, [(stream, slot, req)])
        lat, px_done, n_calls, sizes = [], 0, 0, []
        every = list(self.streams.values()) + list(self.waiting)
        remaining = sum(len(s.queue) for s in every)
        t_first = min((s.queue[0].t_arrival for s in every if s.queue), default=0.0)
        while remaining:
            now = time.perf_counter() - t0
            # admissions (in request order) and closes of finished streams
            while self.waiting and self.waiting[0].queue[0].t_arrival <= now \
                    and self.used + self.waiting[0].need <= self.budget:
                s = self.waiting.popleft()
                self._materialise(s)
                self.admissions.append((s.sid, now))
            for s in list(self.streams.values()):
                if s.close_when_done and not s.queue and not s.uploaded and not s.inflight:
                    self._close_stream(s)
                    self.closes.append((s.sid, now))
            if self.dirty and not inflight:
                self._rebuild()
            # uploads of arrived requests into free slots
            for s in self.streams.values():
                while s.queue and s.queue[0].t_arrival <= now:
                    req = s.queue[0]
                    if req.kind == "keyframe":
                        if s.inflight or s.uploaded:
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
                    s.uploaded.append((slot, req))
            # one call with at most one ready frame per stream (none while the
            # batch waits to be rebuilt over a new set of streams)
            active, imgs, poses, items = [], [], [], []
            if not self.dirty and self.batch is not None and len(inflight) < max_calls_in_flight:
                for sid in sorted(self.streams):
                    s = self.streams[sid]
                    if s.inflight or not s.uploaded:
                        continue
                    slot, req = s.uploaded.popleft()
                    self.compute.wait_event(s.copy_done[slot])
                    active.append(self.member[sid])
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
        for s in list(self.streams.values()):
            if s.close_when_done and not s.queue:
                self._close_stream(s)
                self.closes.append((s.sid, time.perf_counter() - t0))
        if self.dirty:
            self._rebuild()
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
        for s in list(self.streams.values()):
            if s.kf is not None:
                s.kf.close()
