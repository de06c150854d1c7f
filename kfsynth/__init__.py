"""Seeded synthetic inputs for the per-frame keyframe depth update.

This module draws scenes, camera trajectories, rendered images and noisy
network-style priors. It holds none of the depth-update method's arithmetic
(no epipolar search, no filter, no fusion): both the CPU oracle and the GPU
library consume what it produces, and neither is imported here.

Scenes stand in for the indoor sequences (depth roughly 0.5-5 m) the paper
evaluates on (Sec. III); no dataset item is reproduced.
"""

from .scene import (  # noqa: F401
    camera_matrix,
    Scene,
    make_scene,
    render,
    so3_exp,
    pose_matrix,
    Priors,
    make_priors,
    KeyframeCase,
    make_case,
    CONFIGS,
    config_case,
    seed_for,
)
