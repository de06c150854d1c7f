"""ctypes binding of include/kf.h (argument marshalling only).

Every step of the depth update runs in the HIP library ``libkf.so``; this
module checks shapes and dtypes, hands device pointers and the current HIP
stream to the C ABI, and raises ``KfError`` on a non-zero status. PyTorch
supplies device memory and streams. If the library is not built, loading
fails loudly (there is no fallback path).
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_size_t, c_void_p
from typing import Optional

import numpy as np

LIB_PATH = os.environ.get("KF_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkf.so")

KF_OK = 0
KF_ERR_ARG = -1
KF_ERR_OOM = -2
KF_ERR_HIP = -3
KF_ERR_STATE = -4
KF_ERR_INPUT = -5
KF_ERR_TIMEOUT = -6

KF_F64 = 0
KF_F32 = 1
KF_BF16_F32 = 2
PRECISIONS = {"f64": KF_F64, "f32": KF_F32, "bf16": KF_BF16_F32}

KF_VARIANT_FULL = 0
KF_VARIANT_NO_PAIRWISE = 1
KF_VARIANT_SCALE_POSTFIT = 2
VARIANTS = {"full": KF_VARIANT_FULL, "no_pairwise": KF_VARIANT_NO_PAIRWISE, "scale_postfit": KF_VARIANT_SCALE_POSTFIT}

KF_PAT_LINE5 = 0
KF_PAT_SQ5X5 = 1
PATTERNS = {"line5": KF_PAT_LINE5, "sq5x5": KF_PAT_SQ5X5}


class KfConfig(ctypes.Structure):
    _fields_ = [
        ("width", c_int32), ("height", c_int32),
        ("fx", c_double), ("fy", c_double), ("cx", c_double), ("cy", c_double),
        ("n_samples", c_int32), ("pattern", c_int32),
        ("n_gn", c_int32), ("n_cg", c_int32),
        ("cg_rtol", c_double), ("cg_max", c_int32), ("cg_variant", c_int32),
        ("huber_delta", c_double),
        ("d_near", c_double), ("d_far", c_double),
        ("grad_gate", c_double), ("sigma_photo", c_double), ("r_floor", c_double),
        ("precision", c_int32),
        ("solver_tiles_x", c_int32), ("solver_tiles_y", c_int32),
        ("solver_threads", c_int32), ("solver_cooperative", c_int32), ("pipeline_frames", c_int32),
        ("variant", c_int32), ("robust", c_int32), ("lambda_trans", c_double), ("lambda_inliers", c_int32),
        ("solver_timeout_ms", c_double),
        ("stream", c_void_p), ("workspace", c_void_p), ("workspace_bytes", c_size_t),
    ]


class KfFrameStats(ctypes.Structure):
    _fields_ = [
        ("n_searched", c_int32), ("n_updated", c_int32), ("n_valid", c_int32), ("cg_iterations", c_int32),
        ("scale", c_double), ("cg_rel_residual", c_double), ("team_syncs", c_int32), ("new_keyframe", c_int32),
    ]


class KfBatchConfig(ctypes.Structure):
    _fields_ = [
        ("stream", c_void_p), ("use_graph", c_int32), ("workspace", c_void_p), ("workspace_bytes", c_size_t),
    ]


KF_BATCH_MAX_MEMBERS = 256


class KfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None):
    """Loads libkf.so once; raises if it is missing (build it with paper_2207_12244_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libkf.so not found at {p}; build it with `python -m paper_2207_12244_amd.build`")
    lib = ctypes.CDLL(p)
    P = c_void_p
    dbl16 = POINTER(c_double)
    sig = {
        "kf_config_default": (None, [POINTER(KfConfig), c_int32, c_int32]),
        "kf_workspace_bytes": (c_size_t, [POINTER(KfConfig)]),
        "kf_create": (c_int32, [POINTER(KfConfig), POINTER(P)]),
        "kf_destroy": (None, [P]),
        "kf_last_error": (c_char_p, [P]),
        "kf_status_string": (c_char_p, [c_int32]),
        "kf_set_prior": (c_int32, [P, P, P, P, P, P, P, P, dbl16]),
        "kf_set_prior_network": (c_int32, [P, P, P, P, P, P, P, P, c_int32, c_int32, c_double, dbl16]),
        "kf_stereo_update": (c_int32, [P, P, dbl16]),
        "kf_solve": (c_int32, [P]),
        "kf_fuse_frame": (c_int32, [P, P, dbl16]),
        "kf_fuse_frame_static": (c_int32, [P, P, dbl16]),
        "kf_read_depth": (c_int32, [P, P, P, POINTER(c_double)]),
        "kf_read_stats": (c_int32, [P, POINTER(KfFrameStats)]),
        "kf_export_state": (c_int32, [P, P, P, P, P, POINTER(c_double)]),
        "kf_solver_layout": (c_int32, [P, POINTER(c_int32)]),
        "kf_solve_stream": (c_void_p, [P]),
        "kf_probe_sync": (c_int32, [P, c_int32, c_int32]),
        "kf_import_state": (c_int32, [P, P, P, P, POINTER(c_double)]),
        "kf_batch_config_default": (None, [POINTER(KfBatchConfig)]),
        "kf_batch_workspace_bytes": (c_size_t, [POINTER(P), c_int32]),
        "kf_batch_create": (c_int32, [POINTER(P), c_int32, POINTER(KfBatchConfig), POINTER(P)]),
        "kf_batch_fuse": (c_int32, [P, POINTER(P), POINTER(c_double)]),
        "kf_batch_fuse_subset": (c_int32, [P, c_int32, POINTER(c_int32), POINTER(P), POINTER(c_double)]),
        "kf_batch_stereo_update": (c_int32, [P, POINTER(P), POINTER(c_double)]),
        "kf_batch_solve": (c_int32, [P]),
        "kf_batch_layout": (c_int32, [P, POINTER(c_int32)]),
        "kf_batch_last_error": (c_char_p, [P]),
        "kf_batch_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


EXPORTED_SYMBOLS = (
    "kf_config_default", "kf_workspace_bytes", "kf_create", "kf_destroy", "kf_last_error", "kf_status_string",
    "kf_set_prior", "kf_set_prior_network", "kf_stereo_update", "kf_solve", "kf_fuse_frame", "kf_fuse_frame_static", "kf_read_depth",
    "kf_read_stats",
    "kf_export_state", "kf_import_state", "kf_solver_layout", "kf_solve_stream", "kf_probe_sync",
    "kf_batch_config_default", "kf_batch_workspace_bytes", "kf_batch_create", "kf_batch_fuse",
    "kf_batch_fuse_subset", "kf_batch_stereo_update", "kf_batch_solve", "kf_batch_layout",
    "kf_batch_last_error", "kf_batch_destroy",
)


def status_string(status: int) -> str:
    try:
        return load_library().kf_status_string(int(status)).decode()
    except RuntimeError:
        return str(status)


# ---------------------------------------------------------------- same-name wrappers

def kf_config_default(width: int, height: int) -> KfConfig:
    cfg = KfConfig()
    load_library().kf_config_default(ctypes.byref(cfg), int(width), int(height))
    return cfg


def kf_workspace_bytes(cfg: KfConfig) -> int:
    return int(load_library().kf_workspace_bytes(ctypes.byref(cfg)))


def _check(status: int, ctx=None):
    if status != KF_OK:
        msg = load_library().kf_last_error(ctx).decode() if ctx else ""
        raise KfError(status, msg)


def _pose(T) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(4, 4))
    return (c_double * 16)(*a.ravel().tolist())


def kf_create(cfg: KfConfig):
    h = c_void_p()
    st = load_library().kf_create(ctypes.byref(cfg), ctypes.byref(h))
    if st != KF_OK:
        raise KfError(st, "kf_create rejected the configuration or workspace")
    return h


def kf_destroy(ctx) -> None:
    load_library().kf_destroy(ctx)


def kf_set_prior(ctx, image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var, T_wc0) -> None:
    _check(load_library().kf_set_prior(ctx, image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y,
                                       grad_y_var, _pose(T_wc0)), ctx)


def kf_set_prior_network(ctx, image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var, net_width,
                         net_height, focal_ref, T_wc0) -> None:
    _check(load_library().kf_set_prior_network(ctx, image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y,
                                               grad_y_var, int(net_width), int(net_height), float(focal_ref),
                                               _pose(T_wc0)), ctx)


def kf_stereo_update(ctx, image1, T_wc1) -> None:
    _check(load_library().kf_stereo_update(ctx, image1, _pose(T_wc1)), ctx)


def kf_solve(ctx) -> None:
    _check(load_library().kf_solve(ctx), ctx)


def kf_fuse_frame(ctx, image1, T_wc1) -> None:
    _check(load_library().kf_fuse_frame(ctx, image1, _pose(T_wc1)), ctx)


def kf_read_depth(ctx, depth_out, var_out=None) -> float:
    s = c_double(0.0)
    _check(load_library().kf_read_depth(ctx, depth_out, var_out, ctypes.byref(s)), ctx)
    return s.value


def kf_read_stats(ctx) -> KfFrameStats:
    st = KfFrameStats()
    _check(load_library().kf_read_stats(ctx, ctypes.byref(st)), ctx)
    return st


def kf_export_state(ctx, x=None, rho=None, rho_var=None, match=None) -> float:
    t = c_double(0.0)
    _check(load_library().kf_export_state(ctx, x, rho, rho_var, match, ctypes.byref(t)), ctx)
    return t.value


def kf_solver_layout(ctx):
    out = (c_int32 * 5)()
    _check(load_library().kf_solver_layout(ctx, out), ctx)
    return dict(tiles_x=out[0], tiles_y=out[1], tile_w=out[2], tile_h=out[3], threads=out[4])


def kf_import_state(ctx, x=None, rho=None, rho_var=None, tau: Optional[float] = None) -> None:
    tp = ctypes.byref(c_double(float(tau))) if tau is not None else None
    _check(load_library().kf_import_state(ctx, x, rho, rho_var, tp), ctx)


def _bcheck(status: int, batch=None):
    if status != KF_OK:
        msg = load_library().kf_batch_last_error(batch).decode() if batch else ""
        raise KfError(status, msg)


def _ctx_array(ctxs):
    arr = (c_void_p * len(ctxs))()
    for i, c in enumerate(ctxs):
        arr[i] = c.value if isinstance(c, c_void_p) else c
    return arr


def kf_batch_config_default() -> KfBatchConfig:
    cfg = KfBatchConfig()
    load_library().kf_batch_config_default(ctypes.byref(cfg))
    return cfg


def kf_batch_workspace_bytes(ctxs) -> int:
    arr = _ctx_array(ctxs)
    return int(load_library().kf_batch_workspace_bytes(arr, len(ctxs)))


def kf_batch_create(ctxs, cfg: KfBatchConfig):
    out = c_void_p()
    arr = _ctx_array(ctxs)
    _check(load_library().kf_batch_create(arr, len(ctxs), ctypes.byref(cfg), ctypes.byref(out)))
    return out


def _frame_args(images, poses):
    n = len(images)
    arr = (c_void_p * n)()
    for i, p in enumerate(images):
        arr[i] = p.value if isinstance(p, c_void_p) else p
    P = np.ascontiguousarray(np.stack([np.asarray(T, dtype=np.float64).reshape(4, 4) for T in poses]), np.float64)
    return arr, P


def kf_batch_fuse(batch, images, poses) -> None:
    """images: sequence of device pointers (int or c_void_p); poses: sequence of 4x4 matrices."""
    arr, P = _frame_args(images, poses)
    _bcheck(load_library().kf_batch_fuse(batch, arr, P.ctypes.data_as(POINTER(c_double))), batch)


def kf_batch_fuse_subset(batch, members, images, poses) -> None:
    """members: indices into the batch; images / poses: one per listed member."""
    if len(members) == 0:
        return
    arr, P = _frame_args(images, poses)
    idx = (c_int32 * len(members))(*[int(i) for i in members])
    _bcheck(load_library().kf_batch_fuse_subset(batch, len(members), idx, arr,
                                                P.ctypes.data_as(POINTER(c_double))), batch)


def kf_batch_stereo_update(batch, images, poses) -> None:
    arr, P = _frame_args(images, poses)
    _bcheck(load_library().kf_batch_stereo_update(batch, arr, P.ctypes.data_as(POINTER(c_double))), batch)


def kf_batch_solve(batch) -> None:
    _bcheck(load_library().kf_batch_solve(batch), batch)


def kf_batch_layout(batch):
    out = (c_int32 * 4)()
    _bcheck(load_library().kf_batch_layout(batch, out), batch)
    return dict(workgroups=out[0], threads=out[1], ppt=out[2], max_queue=out[3])


def kf_batch_destroy(batch) -> None:
    load_library().kf_batch_destroy(batch)


# ---------------------------------------------------------------- torch convenience layer

def _torch():
    import torch
    return torch


class Keyframe:
    """One keyframe context with a torch-allocated workspace on the current device.

    Maps are torch tensors of the form's element type (float64 for "f64",
    float32 otherwise), images uint8; all H x W, contiguous, on the GPU.
    """

    def __init__(self, width: int, height: int, *, precision: str = "f32", pattern: str = "line5",
                 n_samples: int = 32, n_gn: int = 10, n_cg: int = 20, cg_rtol: float = 0.0, cg_max: int = 4000,
                 huber_delta: float = 1.345, d_near: float = 0.4, d_far: float = 10.0, grad_gate: float = 6.0,
                 sigma_photo: float = 1.0, r_floor: float = 1e-6, K=None, tiles=(0, 0), solver_threads: int = 0,
                 cooperative: bool = False, cg_variant: str = "auto", solver_timeout_ms: float = 0.0,
                 pipeline_frames: bool = False, variant: str = "full", robust: str = "huber", lambda_trans: float = 0.0,
                 lambda_inliers: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Keyframe needs a GPU (the library has no CPU path)")
        cfg = kf_config_default(width, height)
        if K is not None:
            K = np.asarray(K, dtype=np.float64)
            cfg.fx, cfg.fy, cfg.cx, cfg.cy = float(K[0, 0]), float(K[1, 1]), float(K[0, 2]), float(K[1, 2])
        cfg.precision = PRECISIONS[precision]
        cfg.pattern = PATTERNS[pattern]
        cfg.n_samples, cfg.n_gn, cfg.n_cg = int(n_samples), int(n_gn), int(n_cg)
        cfg.cg_rtol, cfg.cg_max = float(cg_rtol), int(cg_max)
        cfg.huber_delta, cfg.d_near, cfg.d_far = float(huber_delta), float(d_near), float(d_far)
        cfg.grad_gate, cfg.sigma_photo, cfg.r_floor = float(grad_gate), float(sigma_photo), float(r_floor)
        cfg.solver_tiles_x, cfg.solver_tiles_y = int(tiles[0]), int(tiles[1])
        cfg.solver_threads, cfg.solver_cooperative = int(solver_threads), int(bool(cooperative))
        cfg.cg_variant = {"auto": 0, "textbook": 1, "pipelined": 2}[cg_variant]
        cfg.solver_timeout_ms = float(solver_timeout_ms)
        cfg.pipeline_frames = int(bool(pipeline_frames))
        cfg.variant = VARIANTS[variant]
        cfg.robust = {"huber": 0, "tukey": 1}[robust]
        cfg.lambda_trans, cfg.lambda_inliers = float(lambda_trans), int(lambda_inliers)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg.stream = c_void_p(self.stream.cuda_stream)
        nbytes = kf_workspace_bytes(cfg)
        if nbytes == 0:
            raise KfError(KF_ERR_ARG, "invalid configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        cfg.workspace = c_void_p(aligned)
        cfg.workspace_bytes = nbytes
        self.cfg = cfg
        self.W, self.H = int(width), int(height)
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.ctx = kf_create(cfg)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            kf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _map(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.dtype != self.dtype or tuple(t.shape) != (self.H, self.W) \
                or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor of shape ({self.H}, {self.W})")
        return c_void_p(t.data_ptr())

    def _img(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or tuple(t.shape) != (self.H, self.W) \
                or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous uint8 CUDA tensor of shape ({self.H}, {self.W})")
        return c_void_p(t.data_ptr())

    def set_prior(self, image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var, T_wc0):
        self._keep = (image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var)
        kf_set_prior(self.ctx, self._img(image0, "image0"), self._map(logdepth, "logdepth"),
                     self._map(logdepth_var, "logdepth_var"), self._map(grad_x, "grad_x"),
                     self._map(grad_x_var, "grad_x_var"), self._map(grad_y, "grad_y"),
                     self._map(grad_y_var, "grad_y_var"), T_wc0)

    def set_prior_network(self, image0, logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var, T_wc0,
                          focal_ref: float):
        """New keyframe from the network's six maps at the network's own size
        (all of one shape Hn x Wn), resampled and focal-shifted in the library."""
        torch = _torch()
        maps = (logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var)
        shape = tuple(logdepth.shape) if isinstance(logdepth, torch.Tensor) else None
        for name, t in zip(("logdepth", "logdepth_var", "grad_x", "grad_x_var", "grad_y", "grad_y_var"), maps):
            if not isinstance(t, torch.Tensor) or t.dtype != self.dtype or t.dim() != 2 or tuple(t.shape) != shape \
                    or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor, all six of one 2-D shape")
        self._keep = (image0, *maps)
        kf_set_prior_network(self.ctx, self._img(image0, "image0"), *[c_void_p(t.data_ptr()) for t in maps],
                             shape[1], shape[0], focal_ref, T_wc0)

    def _hold(self, image1):
        # the library reads image1 when the stream reaches the call: keep the
        # caching allocator from handing its memory out before then
        if image1.device.type == "cuda":
            image1.record_stream(self.stream)

    def stereo_update(self, image1, T_wc1):
        kf_stereo_update(self.ctx, self._img(image1, "image1"), T_wc1)
        self._hold(image1)

    def solve(self):
        kf_solve(self.ctx)

    def fuse_frame(self, image1, T_wc1):
        kf_fuse_frame(self.ctx, self._img(image1, "image1"), T_wc1)
        self._hold(image1)

    def read_depth(self, with_var: bool = False):
        torch = _torch()
        d = torch.empty((self.H, self.W), dtype=self.dtype, device="cuda")
        v = torch.empty((self.H, self.W), dtype=self.dtype, device="cuda") if with_var else None
        s = kf_read_depth(self.ctx, c_void_p(d.data_ptr()), c_void_p(v.data_ptr()) if v is not None else None)
        return (d, s, v) if with_var else (d, s)

    def solver_layout(self):
        return kf_solver_layout(self.ctx)

    def solve_stream(self):
        """torch stream the solves run on (pipeline_frames), else the context's stream."""
        torch = _torch()
        h = load_library().kf_solve_stream(self.ctx)
        return torch.cuda.ExternalStream(h) if h else self.stream

    def stats(self) -> KfFrameStats:
        return kf_read_stats(self.ctx)

    def probe_sync(self, rounds: int, nvalues: int = 2) -> None:
        """Enqueues the team-synchronisation probe (kf_probe_sync) on the context's stream."""
        _check(load_library().kf_probe_sync(self.ctx, int(rounds), int(nvalues)), self.ctx)

    def export_state(self):
        torch = _torch()
        x = torch.empty((self.H, self.W), dtype=self.dtype, device="cuda")
        rho = torch.empty_like(x)
        var = torch.empty_like(x)
        match = torch.empty((self.H, self.W), dtype=torch.int32, device="cuda")
        tau = kf_export_state(self.ctx, c_void_p(x.data_ptr()), c_void_p(rho.data_ptr()), c_void_p(var.data_ptr()),
                              c_void_p(match.data_ptr()))
        return dict(x=x, rho=rho, var=var, match=match, tau=tau)

    def import_state(self, x=None, rho=None, var=None, tau=None):
        kf_import_state(self.ctx,
                        self._map(x, "x") if x is not None else None,
                        self._map(rho, "rho") if rho is not None else None,
                        self._map(var, "var") if var is not None else None,
                        tau)


class Batch:
    """Fuses one frame into each of several Keyframe objects with one staging,
    one stereo and one persistent solver launch (replayed as a HIP graph).

    Members must share precision, pattern, n_samples, the solver workgroup
    size, the CG variant and the stream; each keeps its own size and tiling,
    and its results equal those of fusing it alone.
    """

    def __init__(self, keyframes, *, use_graph: bool = True):
        torch = _torch()
        self.members = list(keyframes)
        if not self.members:
            raise ValueError("a batch needs at least one keyframe")
        streams = {kf.stream.cuda_stream for kf in self.members}
        if len(streams) != 1:
            raise ValueError("batch members must share one stream")
        self.stream = self.members[0].stream
        ctxs = [kf.ctx for kf in self.members]
        nbytes = kf_batch_workspace_bytes(ctxs)
        if nbytes == 0:
            raise KfError(KF_ERR_ARG, "invalid batch members")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        cfg = kf_batch_config_default()
        cfg.stream = c_void_p(self.stream.cuda_stream)
        cfg.use_graph = int(bool(use_graph))
        cfg.workspace = c_void_p((self.workspace.data_ptr() + 255) & ~255)
        cfg.workspace_bytes = nbytes
        self.cfg = cfg
        self.batch = kf_batch_create(ctxs, cfg)

    def fuse(self, images, poses):
        kf_batch_fuse(self.batch, self._ptrs(images, poses), poses)

    def _ptrs(self, images, poses):
        if len(images) != len(self.members) or len(poses) != len(self.members):
            raise ValueError(f"need {len(self.members)} images and poses")
        self._keep = list(images)
        return [kf._img(im, f"images[{i}]") for i, (kf, im) in enumerate(zip(self.members, images))]

    def stereo_update(self, images, poses):
        kf_batch_stereo_update(self.batch, self._ptrs(images, poses), poses)

    def fuse_subset(self, members, images, poses):
        """Fuses images[k] / poses[k] into member members[k]; the others are untouched."""
        if len(images) != len(members) or len(poses) != len(members):
            raise ValueError("need one image and pose per listed member")
        ptrs = [self.members[i]._img(im, f"images[{k}]") for k, (i, im) in enumerate(zip(members, images))]
        self._keep = list(images)
        kf_batch_fuse_subset(self.batch, members, ptrs, poses)

    def solve(self):
        kf_batch_solve(self.batch)

    def layout(self):
        return kf_batch_layout(self.batch)

    def close(self):
        if getattr(self, "batch", None) is not None:
            kf_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
