"""Autotuner host logic (no GPU): candidate tile grids obey the library's tiling
rules and are the fewest tiles of the capped size."""

import ctypes
import os

import pytest

from paper_2207_12244_amd import autotune


def _lib():
    from paper_2207_12244_amd import kf
    if not os.path.exists(kf.LIB_PATH):
        pytest.skip("libkf.so not built")
    return kf


@pytest.mark.parametrize("W,H", [(160, 120), (320, 240), (512, 384), (640, 480), (200, 130), (64, 48)])
@pytest.mark.parametrize("threads,ppt", autotune.CANDIDATES)
def test_candidate_tilings_are_valid_and_minimal(W, H, threads, ppt):
    kf = _lib()
    t = autotune.tiles_for(W, H, threads, ppt)
    assert t is not None
    tx, ty = t
    tw, th = -(-W // tx), -(-H // ty)
    assert tw * th <= threads * ppt and tx * ty <= autotune.MAX_TEAM
    cfg = kf.kf_config_default(W, H)
    cfg.precision = kf.KF_BF16_F32
    cfg.solver_threads = threads
    cfg.solver_tiles_x, cfg.solver_tiles_y = tx, ty
    assert kf.kf_workspace_bytes(cfg) > 0
    # no grid with fewer tiles fits the cap
    for n in range(1, tx * ty):
        for a in range(1, n + 1):
            if n % a:
                continue
            b = n // a
            assert -(-W // a) * -(-H // b) > threads * ppt or -(-W // a) + -(-H // b) > threads


def test_cache_key_is_order_free():
    k1 = autotune.cache_key([(640, 480), (160, 120), (640, 480)], "bf16", 10, 20, "dev")
    k2 = autotune.cache_key([(160, 120), (640, 480), (640, 480)], "bf16", 10, 20, "dev")
    assert k1 == k2 and "640x480:2" in k1 and "160x120:1" in k1
