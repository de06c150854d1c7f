"""Scene, trajectory, image and prior synthesis (seeded, CPU, numpy).

Recipe (all draws from numpy's PCG64 seeded by ``SeedSequence(seed)``, in the
order written below):

* Camera: pinhole, fx = fy = 0.8 W, cx = W/2, cy = H/2; integer pixel
  coordinates are pixel centres.
* Scene: three infinite planes. Plane j is the canonical frame rotated by
  theta_j ~ U(0, 45 deg) about an axis (cos phi_j, sin phi_j, 0),
  phi_j ~ U(0, 2 pi); its normal is R_j (0, 0, -1) (facing the keyframe camera),
  it passes through (0, 0, d_j) with d_j ~ U(1, 4) m, and its texture axes are
  R_j (1, 0, 0) and R_j (0, 1, 0). The visible surface is the nearest positive
  ray-plane hit; depths are z-depths.
* Texture: 4-octave value noise in each plane's metric 2-D frame, cell size
  L = 0.25 m at octave 0 halving per octave, amplitudes 2^-o normalised to
  sum 1, lattice values U(0, 1) from a splitmix64 chain over
  (texture seed, plane, octave, ix, iy), smoothstep-interpolated. Images are
  rendered with a 2x2 box supersample (offsets +-0.25 px) and stored as
  rint(127.5 + 255 g (V - 1/2)) clipped to [0, 255] in uint8, with contrast
  gain g = 2 so that intensities span the full 0-255 range (about 4 % of
  pixels saturate).
* Acceptance: every pixel of every view has a hit with depth in [0.5, 5] m
  and every plane covers at least 5 % of the keyframe; otherwise the
  trajectory (then the scene) is redrawn.
* Motion "single": one new frame at t = 0.05 u, R = exp(1 deg a), with u, a
  uniform on the unit sphere.  Motion "walk": u_k = normalise(u_{k-1} + 0.3 xi),
  t_k = t_{k-1} + 0.02 u_k, a_k = normalise(a_{k-1} + 0.3 xi'),
  R_k = R_{k-1} exp(0.5 deg a_k), starting from the keyframe at the origin.
* Priors (network stand-ins): log-depth mu = ln z + sigma eps with sigma
  log-uniform in [0.02, 0.3] per pixel; x/y log-depth gradients = forward
  difference of ln z (zero in the last column / row) + sigma_g eps with
  sigma_g log-uniform in [0.01, 0.2]; the variances passed on are sigma^2.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

CONTRAST_GAIN = 2.0

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def _splitmix64(x):
    """splitmix64 finaliser (Steele, Lea and Flood 2014), wrapping uint64."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        return z ^ (z >> np.uint64(31))


def _lattice_prefix(seed: int, plane: int, octave: int) -> np.uint64:
    h = _splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    h = _splitmix64(h ^ np.uint64(plane))
    return _splitmix64(h ^ np.uint64(octave))


def _lattice_u01(prefix: np.uint64, ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    h = _splitmix64(prefix ^ ix.astype(np.int64).view(np.uint64))
    h = _splitmix64(h ^ iy.astype(np.int64).view(np.uint64))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _lattice_lookup(prefix, ix, iy):
    """Lattice values at integer coordinates, via a table over their bounding box."""
    x0, x1 = int(ix.min()), int(ix.max())
    y0, y1 = int(iy.min()), int(iy.max())
    nx, ny = x1 - x0 + 1, y1 - y0 + 1
    if nx * ny > 4_000_000:
        return _lattice_u01(prefix, ix, iy)
    gx, gy = np.meshgrid(np.arange(x0, x1 + 1, dtype=np.int64),
                         np.arange(y0, y1 + 1, dtype=np.int64))
    table = _lattice_u01(prefix, gx, gy)
    return table[iy - y0, ix - x0]


def value_noise(seed: int, plane: int, s: np.ndarray, t: np.ndarray,
                cell: float = 0.25, octaves: int = 4) -> np.ndarray:
    """Fractal value noise in [0, 1] at metric plane coordinates (s, t)."""
    acc = np.zeros_like(s, dtype=np.float64)
    norm = 0.0
    for o in range(octaves):
        amp = 0.5 ** o
        scale = (2.0 ** o) / cell
        u = s * scale
        v = t * scale
        fu_i = np.floor(u)
        fv_i = np.floor(v)
        fu = u - fu_i
        fv = v - fv_i
        su = fu * fu * (3.0 - 2.0 * fu)
        sv = fv * fv * (3.0 - 2.0 * fv)
        iu = fu_i.astype(np.int64)
        iv = fv_i.astype(np.int64)
        pre = _lattice_prefix(seed, plane, o)
        l00 = _lattice_lookup(pre, iu, iv)
        l10 = _lattice_lookup(pre, iu + 1, iv)
        l01 = _lattice_lookup(pre, iu, iv + 1)
        l11 = _lattice_lookup(pre, iu + 1, iv + 1)
        n = (1 - su) * (1 - sv) * l00 + su * (1 - sv) * l10 + (1 - su) * sv * l01 + su * sv * l11
        acc += amp * n
        norm += amp
    return acc / norm


def camera_matrix(W: int, H: int) -> np.ndarray:
    f = 0.8 * W
    return np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])


def so3_exp(w) -> np.ndarray:
    """Rotation matrix of the rotation vector w (Rodrigues)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    if th < 1e-15:
        return np.eye(3)
    k = w / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * (Kx @ Kx)


def pose_matrix(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


@dataclass
class Scene:
    normals: np.ndarray   # (3, 3): row j = unit normal of plane j
    points: np.ndarray    # (3, 3): row j = a point on plane j
    axis_s: np.ndarray    # (3, 3): row j = first in-plane texture axis
    axis_t: np.ndarray    # (3, 3): row j = second in-plane texture axis
    tex_seed: int
    cell: float = 0.25


def make_scene(rng: np.random.Generator, tex_seed: int) -> Scene:
    normals, points, a_s, a_t = [], [], [], []
    for _ in range(3):
        theta = rng.uniform(0.0, math.radians(45.0))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        d = rng.uniform(1.0, 4.0)
        R = so3_exp(theta * np.array([math.cos(phi), math.sin(phi), 0.0]))
        normals.append(R @ np.array([0.0, 0.0, -1.0]))
        a_s.append(R @ np.array([1.0, 0.0, 0.0]))
        a_t.append(R @ np.array([0.0, 1.0, 0.0]))
        points.append(np.array([0.0, 0.0, d]))
    return Scene(np.array(normals), np.array(points), np.array(a_s), np.array(a_t), tex_seed)


def _cast(scene: Scene, K: np.ndarray, T_wc: np.ndarray, u: np.ndarray, v: np.ndarray):
    """Nearest positive ray-plane hit for pixel coordinates (u, v).

    Returns (z-depth, plane index, texture s, texture t); depth is +inf and the
    plane index -1 where no plane is hit in front of the camera.
    """
    fx, fy, cx, cy = K[0, 0], K[1, 1], K[0, 2], K[1, 2]
    R = T_wc[:3, :3]
    c = T_wc[:3, 3]
    rc = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1)
    rw = rc @ R.T
    best = np.full(u.shape, np.inf)
    idx = np.full(u.shape, -1, dtype=np.int64)
    for j in range(3):
        n = scene.normals[j]
        den = rw @ n
        num = float(n @ (scene.points[j] - c))
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = num / den
        ok = (den != 0) & (lam > 0) & (lam < best)
        best = np.where(ok, lam, best)
        idx = np.where(ok, j, idx)
    s = np.zeros(u.shape)
    t = np.zeros(u.shape)
    for j in range(3):
        m = idx == j
        if not np.any(m):
            continue
        P = c + best[m][:, None] * rw[m]
        dP = P - scene.points[j]
        s[m] = dP @ scene.axis_s[j]
        t[m] = dP @ scene.axis_t[j]
    return best, idx, s, t


def render(scene: Scene, K: np.ndarray, T_wc: np.ndarray, W: int, H: int,
           supersample: bool = True):
    """Render one view: (uint8 image, z-depth at pixel centres, plane index)."""
    vv, uu = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    depth, pid, _, _ = _cast(scene, K, T_wc, uu, vv)
    offs = [(-0.25, -0.25), (0.25, -0.25), (-0.25, 0.25), (0.25, 0.25)] if supersample else [(0.0, 0.0)]
    acc = np.zeros((H, W))
    for du, dv in offs:
        _, p2, s, t = _cast(scene, K, T_wc, uu + du, vv + dv)
        val = np.zeros((H, W))
        for j in range(3):
            m = p2 == j
            if np.any(m):
                val[m] = value_noise(scene.tex_seed, j, s[m], t[m], scene.cell)
        acc += val
    vmean = acc / len(offs)
    img = np.clip(np.rint(127.5 + 255.0 * CONTRAST_GAIN * (vmean - 0.5)), 0, 255).astype(np.uint8)
    return img, depth, pid


@dataclass
class Priors:
    logdepth: np.ndarray
    logdepth_var: np.ndarray
    gx: np.ndarray
    gx_var: np.ndarray
    gy: np.ndarray
    gy_var: np.ndarray

    def maps(self):
        return (self.logdepth, self.logdepth_var, self.gx, self.gx_var, self.gy, self.gy_var)


def make_priors(rng: np.random.Generator, depth: np.ndarray) -> Priors:
    H, W = depth.shape
    x = np.log(depth)
    sig = np.exp(rng.uniform(math.log(0.02), math.log(0.3), size=(H, W)))
    mu = x + sig * rng.standard_normal((H, W))
    gxt = np.zeros((H, W))
    gxt[:, :-1] = x[:, 1:] - x[:, :-1]
    sgx = np.exp(rng.uniform(math.log(0.01), math.log(0.2), size=(H, W)))
    gx = gxt + sgx * rng.standard_normal((H, W))
    gyt = np.zeros((H, W))
    gyt[:-1, :] = x[1:, :] - x[:-1, :]
    sgy = np.exp(rng.uniform(math.log(0.01), math.log(0.2), size=(H, W)))
    gy = gyt + sgy * rng.standard_normal((H, W))
    return Priors(mu, sig ** 2, gx, sgx ** 2, gy, sgy ** 2)


# Per-configuration workload description (data only). Keys prefixed with
# "method_" are the depth-update settings the configuration runs with.
CONFIGS = {
    0: dict(name="plain-f64-160x120", sizes=[(160, 120)], frames=1, motion="single",
            precision="f64", pattern="line5", n_samples=32, n_gn=10, n_cg=0, cg_rtol=1e-12,
            cg_max=4000),
    1: dict(name="f32-320x240-seq30", sizes=[(320, 240)], frames=30, motion="walk",
            precision="f32", pattern="sq5x5", n_samples=64, n_gn=10, n_cg=20, cg_rtol=0.0,
            cg_max=20),
    2: dict(name="bf16-640x480-seq30", sizes=[(640, 480)], frames=30, motion="walk",
            precision="bf16", pattern="sq5x5", n_samples=128, n_gn=10, n_cg=20, cg_rtol=0.0,
            cg_max=20),
    3: dict(name="batched-64kf-mixed", sizes=[(160, 120), (320, 240), (512, 384), (640, 480)],
            frames=1, motion="single", keyframes=64, precision="bf16", pattern="line5",
            n_samples=32, n_gn=10, n_cg=20, cg_rtol=0.0, cg_max=20),
    4: dict(name="serving-32streams-mixed", sizes=[(320, 240), (512, 384), (640, 480)],
            frames=20, motion="walk", streams=32, rate_hz=30.0, precision="f32",
            pattern="sq5x5", n_samples=64, n_gn=10, n_cg=20, cg_rtol=0.0, cg_max=20),
}


def seed_for(config: int, case: int) -> int:
    return 1000 * int(config) + int(case)


@dataclass
class KeyframeCase:
    W: int
    H: int
    K: np.ndarray
    scene: Scene
    T_wc0: np.ndarray
    image0: np.ndarray
    depth0: np.ndarray
    priors: Priors
    poses: List[np.ndarray] = field(default_factory=list)     # T_wc of frames 1..F
    images: List[np.ndarray] = field(default_factory=list)
    seed: int = 0
    motion: str = "single"


def _trajectory(rng: np.random.Generator, motion: str, frames: int,
                step_t: Optional[float] = None, step_r_deg: Optional[float] = None,
                translation_scale: float = 1.0) -> List[np.ndarray]:
    poses = []
    if motion == "single":
        st = 0.05 if step_t is None else step_t
        sr = 1.0 if step_r_deg is None else step_r_deg
        for _ in range(frames):
            u = _unit(rng)
            a = _unit(rng)
            poses.append(pose_matrix(so3_exp(math.radians(sr) * a), st * u / translation_scale))
        return poses
    if motion == "walk":
        st = 0.02 if step_t is None else step_t
        sr = 0.5 if step_r_deg is None else step_r_deg
        u = _unit(rng)
        a = _unit(rng)
        t = np.zeros(3)
        R = np.eye(3)
        for _ in range(frames):
            u = u + 0.3 * rng.standard_normal(3)
            u /= np.linalg.norm(u)
            a = a + 0.3 * rng.standard_normal(3)
            a /= np.linalg.norm(a)
            t = t + st * u
            R = R @ so3_exp(math.radians(sr) * a)
            poses.append(pose_matrix(R, t / translation_scale))
        return poses
    raise ValueError(f"unknown motion {motion!r}")


def _depth_ok(depth: np.ndarray) -> bool:
    return bool(np.all(np.isfinite(depth)) and depth.min() >= 0.5 and depth.max() <= 5.0)


def make_case(seed: int, W: int, H: int, frames: int, motion: str = "single",
              step_t: Optional[float] = None, step_r_deg: Optional[float] = None,
              translation_scale: float = 1.0, max_tries: int = 500) -> KeyframeCase:
    """Draw an accepted scene + trajectory + priors for one keyframe.

    ``translation_scale`` divides every camera translation (the scene itself
    is unchanged), which is how a scale-ambiguous pose source looks.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    K = camera_matrix(W, H)
    T0 = np.eye(4)
    # coarse acceptance check on every 4th pixel before the full render
    cu, cv = np.meshgrid(np.arange(0, W, 4, dtype=float), np.arange(0, H, 4, dtype=float))
    for _ in range(max_tries):
        tex_seed = int(rng.integers(0, 2 ** 62))
        scene = make_scene(rng, tex_seed)
        dc, pc, _, _ = _cast(scene, K, T0, cu, cv)
        if not _depth_ok(dc):
            continue
        if min(np.mean(pc == j) for j in range(3)) < 0.05:
            continue
        img0, depth0, pid0 = render(scene, K, T0, W, H)
        if not _depth_ok(depth0) or min(np.mean(pid0 == j) for j in range(3)) < 0.05:
            continue
        for _ in range(20):
            poses = _trajectory(rng, motion, frames, step_t, step_r_deg, translation_scale)
            ok = True
            for T in poses:
                # judge acceptance on the metric trajectory
                Tm = T.copy()
                Tm[:3, 3] *= translation_scale
                dk, _, _, _ = _cast(scene, K, Tm, cu, cv)
                if not _depth_ok(dk):
                    ok = False
                    break
            if not ok:
                continue
            images = []
            for T in poses:
                Tm = T.copy()
                Tm[:3, 3] *= translation_scale
                img, dk, _ = render(scene, K, Tm, W, H)
                if not _depth_ok(dk):
                    ok = False
                    break
                images.append(img)
            if not ok:
                continue
            priors = make_priors(rng, depth0)
            return KeyframeCase(W, H, K, scene, T0, img0, depth0, priors, poses, images, seed, motion)
    raise RuntimeError(f"no acceptable scene for seed {seed} after {max_tries} tries")


def config_case(config: int, case: int = 0, frames: Optional[int] = None,
                size_index: Optional[int] = None, translation_scale: float = 1.0) -> KeyframeCase:
    """The generator case ``case`` of configuration ``config`` (seed 1000*config + case)."""
    cfg = CONFIGS[config]
    seed = seed_for(config, case)
    if size_index is None:
        if len(cfg["sizes"]) == 1:
            size_index = 0
        else:
            pick = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
            size_index = int(pick.integers(0, len(cfg["sizes"])))
    W, H = cfg["sizes"][size_index]
    nf = cfg["frames"] if frames is None else frames
    return make_case(seed, W, H, nf, cfg["motion"], translation_scale=translation_scale)
