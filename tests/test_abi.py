"""C ABI checks that need no GPU: the library loads, exports every declared symbol,
and rejects bad arguments on the host before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kf.h")


def _lib():
    from paper_2207_12244_amd import kf
    if not os.path.exists(kf.LIB_PATH):
        pytest.skip("libkf.so not built (run __graft_entry__.build())")
    return kf, kf.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    kf, lib = _lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(kf.EXPORTED_SYMBOLS)


def test_defaults_follow_the_documented_readings():
    kf, lib = _lib()
    cfg = kf.kf_config_default(640, 480)
    assert (cfg.width, cfg.height) == (640, 480)
    assert cfg.fx == cfg.fy == 512.0 and cfg.cx == 320.0 and cfg.cy == 240.0
    assert cfg.n_gn == 10 and cfg.n_samples == 32 and cfg.pattern == kf.KF_PAT_LINE5
    assert cfg.huber_delta == 1.345 and cfg.d_near == 0.4 and cfg.d_far == 10.0
    assert cfg.grad_gate == 6.0 and cfg.sigma_photo == 1.0 and cfg.r_floor == 1e-6


@pytest.mark.parametrize("field,value", [
    ("width", 4), ("height", 9000), ("n_samples", 48), ("n_samples", 2048), ("pattern", 7), ("n_gn", 0),
    ("n_cg", 0), ("cg_rtol", -1.0), ("huber_delta", 0.0), ("d_near", 20.0), ("sigma_photo", 0.0),
    ("r_floor", 0.0), ("precision", 9), ("fx", float("nan")), ("solver_timeout_ms", -1.0),
    ("solver_timeout_ms", float("inf")), ("solver_threads", 384),
])
def test_invalid_config_rejected(field, value):
    kf, lib = _lib()
    cfg = kf.kf_config_default(160, 120)
    setattr(cfg, field, value)
    assert kf.kf_workspace_bytes(cfg) == 0
    h = ctypes.c_void_p()
    assert lib.kf_create(ctypes.byref(cfg), ctypes.byref(h)) == kf.KF_ERR_ARG
    assert not h.value


def test_workspace_size_and_oom():
    kf, lib = _lib()
    cfg = kf.kf_config_default(160, 120)
    n = kf.kf_workspace_bytes(cfg)
    assert n > 160 * 120 * 4 * 10
    cfg.workspace = ctypes.c_void_p(1 << 20)     # never dereferenced by kf_create
    cfg.workspace_bytes = n - 1
    h = ctypes.c_void_p()
    assert lib.kf_create(ctypes.byref(cfg), ctypes.byref(h)) == kf.KF_ERR_OOM
    cfg.workspace_bytes = n
    cfg.workspace = None
    assert lib.kf_create(ctypes.byref(cfg), ctypes.byref(h)) == kf.KF_ERR_ARG
    f64 = kf.kf_config_default(160, 120)
    f64.precision = kf.KF_F64
    assert kf.kf_workspace_bytes(f64) > n


def test_calls_out_of_order_and_null_arguments():
    kf, lib = _lib()
    cfg = kf.kf_config_default(64, 48)
    cfg.workspace = ctypes.c_void_p(1 << 20)
    cfg.workspace_bytes = kf.kf_workspace_bytes(cfg)
    h = kf.kf_create(cfg)
    try:
        pose = kf._pose([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]])
        assert lib.kf_fuse_frame(h, ctypes.c_void_p(4096), pose) == kf.KF_ERR_STATE
        assert lib.kf_solve(h) == kf.KF_ERR_STATE
        assert lib.kf_read_depth(h, None, None, None) == kf.KF_ERR_STATE
        assert b"before kf_set_prior" in lib.kf_last_error(h)
        assert lib.kf_set_prior(h, None, None, None, None, None, None, None, pose) == kf.KF_ERR_ARG
        bad = kf._pose([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 1, 1]])
        p = ctypes.c_void_p(4096)
        assert lib.kf_set_prior(h, p, p, p, p, p, p, p, bad) == kf.KF_ERR_ARG
    finally:
        kf.kf_destroy(h)
    assert lib.kf_create(None, None) == kf.KF_ERR_ARG
    assert lib.kf_last_error(None) == b"no context"
    assert lib.kf_status_string(kf.KF_ERR_TIMEOUT) == b"KF_ERR_TIMEOUT"


def test_manual_tiling_validated():
    kf, lib = _lib()
    cfg = kf.kf_config_default(160, 120)
    cfg.solver_tiles_x, cfg.solver_tiles_y = 7, 5
    assert kf.kf_workspace_bytes(cfg) > 0
    cfg.solver_tiles_x, cfg.solver_tiles_y = 7, 0
    assert kf.kf_workspace_bytes(cfg) == 0
    cfg.solver_tiles_x, cfg.solver_tiles_y = 1, 1      # 19200 px in one workgroup: too many per thread
    assert kf.kf_workspace_bytes(cfg) == 0


def test_binding_keyword_surface():
    """The torch convenience layer accepts every documented option (checked without a GPU)."""
    import inspect
    from paper_2207_12244_amd.kf import Keyframe
    params = inspect.signature(Keyframe.__init__).parameters
    for name in ("precision", "pattern", "n_samples", "n_gn", "n_cg", "cg_rtol", "cg_max", "huber_delta",
                 "d_near", "d_far", "grad_gate", "sigma_photo", "r_floor", "K", "tiles", "solver_threads",
                 "cooperative", "cg_variant", "solver_timeout_ms", "stream"):
        assert name in params, name
    import ast
    import os as _os
    src = open(_os.path.join(ROOT, "paper_2207_12244_amd", "kf.py")).read()
    ast.parse(src)
    assert "cfg.cg_variant" in src


def _ctx(kf, W, H, **fields):
    cfg = kf.kf_config_default(W, H)
    for k, v in fields.items():
        setattr(cfg, k, v)
    cfg.workspace = ctypes.c_void_p(1 << 20)
    cfg.workspace_bytes = kf.kf_workspace_bytes(cfg)
    assert cfg.workspace_bytes > 0
    return kf.kf_create(cfg)


def test_batch_rejects_incompatible_members_on_the_host():
    kf, lib = _lib()
    a = _ctx(kf, 160, 120, solver_threads=512)
    b = _ctx(kf, 320, 240, solver_threads=512)
    c = _ctx(kf, 160, 120, solver_threads=512, pattern=kf.KF_PAT_SQ5X5)
    d = _ctx(kf, 160, 120, solver_threads=256)
    e = _ctx(kf, 160, 120, solver_threads=512, precision=kf.KF_F64)
    try:
        n = kf.kf_batch_workspace_bytes([a, b])
        assert n > 0
        assert kf.kf_batch_workspace_bytes([]) == 0
        cfg = kf.kf_batch_config_default()
        assert cfg.use_graph == 1
        cfg.workspace = ctypes.c_void_p(1 << 24)
        cfg.workspace_bytes = n
        out = ctypes.c_void_p()
        for members in ([a, c], [a, d], [a, e], [a, a]):
            arr = kf._ctx_array(members)
            assert lib.kf_batch_create(arr, len(members), ctypes.byref(cfg), ctypes.byref(out)) == kf.KF_ERR_ARG
            assert not out.value
        arr = kf._ctx_array([a, b])
        cfg.workspace_bytes = n - 1
        assert lib.kf_batch_create(arr, 2, ctypes.byref(cfg), ctypes.byref(out)) == kf.KF_ERR_OOM
        cfg.workspace_bytes = n
        cfg.workspace = ctypes.c_void_p((1 << 24) + 8)
        assert lib.kf_batch_create(arr, 2, ctypes.byref(cfg), ctypes.byref(out)) == kf.KF_ERR_ARG
        cfg.workspace = ctypes.c_void_p(1 << 24)
        cfg.use_graph = 2
        assert lib.kf_batch_create(arr, 2, ctypes.byref(cfg), ctypes.byref(out)) == kf.KF_ERR_ARG
        assert lib.kf_batch_create(arr, 0, ctypes.byref(cfg), ctypes.byref(out)) == kf.KF_ERR_ARG
        assert lib.kf_batch_fuse(None, None, None) == kf.KF_ERR_ARG
        assert lib.kf_batch_last_error(None) == b"no batch"
        lib.kf_batch_destroy(None)
    finally:
        for h in (a, b, c, d, e):
            kf.kf_destroy(h)
