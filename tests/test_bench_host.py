"""Host-side logic of bench.py (no GPU): the refusal of several GPUs, the
algorithmic byte count of a solve, the comment-blind source hash that keys the
committed counter summaries, and the loader that drops a summary taken for
another solver source or launch layout."""

import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


@pytest.mark.parametrize("mode", ["--sync-sweep", "--accuracy"])
def test_gpu_modes_need_a_gpu(mode):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert bench.main([mode]) == 2


def test_algorithmic_bytes_of_the_headline_solve():
    # (23 + 9 n_cg) words per pixel per GN iteration, FP32 words
    assert bench.solver_bytes_per_frame(640 * 480, 10, 20) == 10 * (23 + 180) * 4 * 640 * 480 == 2494464000


def test_source_hash_ignores_comments_and_blank_space(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;\n}\n")
    b.write_text("// header\nint f(int x) {   /* inline\n comment */\n\n  return x + 1;  // trailing\n}\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.source_hash(str(a)) == bench.source_hash(str(b))
    assert bench.source_hash(str(a)) != bench.source_hash(str(c))


def test_traffic_summary_is_dropped_for_another_source_or_layout(tmp_path):
    layout = {"tiles_x": 16, "tiles_y": 16, "tile_w": 40, "tile_h": 30, "threads": 512}
    path = tmp_path / "traffic.json"
    good = {"solver_source_sha256_16": bench.source_hash(*bench.SOLVER_SRCS), "hbm_bytes_per_launch": 123,
            "launch_layout": layout}
    path.write_text(json.dumps(good))
    assert bench.load_traffic(str(path), layout) == 123
    assert bench.load_traffic(str(path), dict(layout, threads=256)) is None
    path.write_text(json.dumps(dict(good, solver_source_sha256_16="0" * 16)))
    assert bench.load_traffic(str(path), layout) is None
    assert bench.load_traffic(str(tmp_path / "missing.json"), layout) is None
