"""Seeded synthetic scenes, cameras and target images.

This module only draws random numbers and packs them into arrays.  It holds
none of the rendering method's arithmetic, so both the FP64 oracle and the HIP
path may use it as their common source of inputs.

Workloads (the paper's Appendix A measures 100k random primitives in a volume
with random MLP weights; the dataset cameras are not available, so these
seeded scenes stand in for it):

  C1  1 camera 64x64, 256 primitives, N=8, constant RGB
  C2  1 camera 1280x720, 50k primitives, N=16, colour MLP width 16 depth 2
  C3  1 camera 1920x1080, 200k primitives, N=16, colour MLP width 32 depth 2
  C4  16 cameras (4x640x480, 8x1280x720, 4x1920x1080), 200k primitives,
      N=16, colour MLP width 32 depth 2
  C5  32 cameras 1600x900, 1M primitives, N=32, colour MLP width 32 depth 3

Primitive distributions: centres U[-1,1]^3 (C5: N(0,0.6^2) clipped to
[-2,2]^3), scales log-uniform in [0.02,0.2] (C5: [0.005,0.1]), quaternions
uniform on S^3 (normalised Gaussian, stored un-normalised), W1 ~ U(-1/3,1/3),
b1 ~ U(-pi,pi), W2 ~ U(0,1/8), b2 = 0, omega0 = 10.  Colour-MLP weights and
biases ~ U(+-1/sqrt(fan_in)), xi ~ N(0,1).

  A   8 cameras 800x800, 100k primitives, N=8, omega0=30, degree-3 SH colour
  G   A's scene as Gaussians (standard deviations a third of A's scales)

Opacity (Gaussians only) ~ U(0.2, 0.9).  Temporal weights W_t (time-conditioned
density only) ~ U(-pi, pi); the scene's time xi_t defaults to 0.

Seeds: scene seed 0 (draw order: centres, scales, quats, W1, b1, W2, colours,
SH coefficients or colour-MLP weights, xi, opacity, W_t), camera seed 1, target
seed 2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SCENE_SEED = 0
CAMERA_SEED = 1
TARGET_SEED = 2

XI_DIM = 8  # auxiliary per-primitive colour-MLP input


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    A world point X maps to camera coordinates R @ X + t; a pixel (i, j)
    (column i, row j) has its centre at (i + 0.5, j + 0.5).
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3,3) float32, world -> camera
    t: np.ndarray  # (3,)  float32
    light: Optional[np.ndarray] = None  # (3,) float32 world position of the view's light (relighting colour)


@dataclasses.dataclass
class SceneConfig:
    name: str
    n_prims: int
    n_hidden: int                   # N, width of the density MLP
    cams: List[tuple]               # list of (width, height)
    color_mode: int                 # 0 constant RGB, 1 colour MLP, 2 spherical harmonics (degree 3),
                                    # 3 relighting colour (c_dc + colour MLP of view and light direction),
                                    # 4 per-ray relighting colour (c_dc + colour MLP of entry point, ray and light direction)
    cmlp_width: int = 0
    cmlp_depth: int = 0             # number of hidden layers
    omega0: float = 10.0
    center_dist: str = "uniform"    # "uniform" U[-1,1]^3 or "normal06" N(0,.6^2) clipped
    scale_lo: float = 0.02
    scale_hi: float = 0.2
    backward: bool = True
    primitive: int = 0              # 0 neural primitive, 1 Gaussian (scales are standard deviations)
    temporal: bool = False          # time-conditioned density: a temporal weight W_t per hidden unit
    time: float = 0.0               # the scene's time xi_t (with temporal weights)


CONFIGS = {
    "C1": SceneConfig("C1", 256, 8, [(64, 64)], 0),
    "C2": SceneConfig("C2", 50_000, 16, [(1280, 720)], 1, 16, 2, backward=False),
    "C3": SceneConfig("C3", 200_000, 16, [(1920, 1080)], 1, 32, 2),
    "C4": SceneConfig("C4", 200_000, 16,
                      [(640, 480)] * 4 + [(1280, 720)] * 8 + [(1920, 1080)] * 4,
                      1, 32, 2),
    "C5": SceneConfig("C5", 1_000_000, 32, [(1600, 900)] * 32, 1, 32, 3,
                      center_dist="normal06", scale_lo=0.005, scale_hi=0.1),
    # the 16-view step with the per-ray relighting colour (colour mode 4: one
    # hidden layer of 16 units, a point light per view) instead of the
    # per-(primitive, view) colour network
    "R": SceneConfig("R", 200_000, 16,
                     [(640, 480)] * 4 + [(1280, 720)] * 8 + [(1920, 1080)] * 4,
                     4, 16, 1),
    # the 16-view step with the relighting colour evaluated once per
    # (primitive, view) (colour mode 3: c_dc + colour network of the view
    # direction, the light direction and xi, W32 D2, a point light per view)
    "L": SceneConfig("L", 200_000, 16,
                     [(640, 480)] * 4 + [(1280, 720)] * 8 + [(1920, 1080)] * 4,
                     3, 32, 2),
    # the dynamic-scene application at the 16-view scale: time-conditioned
    # density (a temporal weight per hidden unit) and degree-3 SH colour
    # whose zero-order coefficient follows the polynomial and Fourier terms
    # of the time, at xi_t = 0.5
    "D": SceneConfig("D", 200_000, 16,
                     [(640, 480)] * 4 + [(1280, 720)] * 8 + [(1920, 1080)] * 4,
                     2, temporal=True, time=0.5),
    # stand-in for the paper's throughput protocol (App. A): 100k random
    # primitives in a volume, N = 8, omega0 = 30, degree-3 SH colour, square
    # 800x800 views around the volume; forward only
    "A": SceneConfig("A", 100_000, 8, [(800, 800)] * 8, 2, omega0=30.0, backward=False),
    # the same scene as Gaussians (the paper's 3DGS comparison): the same
    # uniform draws with a third of the scales, so that the 3-sigma ellipsoid
    # of each Gaussian is the bound of the neural primitive it replaces
    "G": SceneConfig("G", 100_000, 8, [(800, 800)] * 8, 2, omega0=30.0, backward=False,
                     scale_lo=0.02 / 3.0, scale_hi=0.2 / 3.0, primitive=1),
}


def cmlp_param_count(width: int, depth: int, n_in: int = 3 + XI_DIM) -> int:
    """Number of colour-MLP parameters: depth hidden ReLU layers of `width`
    units, then a 3-unit output layer; each layer stores W (out x in) then b."""
    if depth <= 0:
        return 0
    n = n_in * width + width
    n += (depth - 1) * (width * width + width)
    n += width * 3 + 3
    return n


def look_at_camera(width: int, height: int, position: np.ndarray,
                   fov_x_deg: float = 60.0) -> Camera:
    """Camera at `position` looking at the origin with a horizontal field of
    view `fov_x_deg`; fx = fy = W / (2 tan(fov/2)), principal point at the
    image centre."""
    p = np.asarray(position, dtype=np.float64)
    fwd = -p / np.linalg.norm(p)
    up_ref = np.array([0.0, 0.0, 1.0])
    if abs(float(fwd @ up_ref)) > 0.999:
        up_ref = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up_ref)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-(R.astype(np.float64) @ p)).astype(np.float32)
    f = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return Camera(width, height, float(np.float32(f)), float(np.float32(f)),
                  float(np.float32(width / 2.0)), float(np.float32(height / 2.0)), R, t)


def make_cameras(sizes, seed: int = CAMERA_SEED, radius: float = 3.0, lights: bool = False) -> List[Camera]:
    """One camera per (width, height), each on the sphere of `radius` at a
    uniformly random direction, looking at the origin.  With `lights`, each
    view also gets a point light at a uniformly random direction on the
    sphere of radius 4 (drawn after all the cameras)."""
    rng = np.random.default_rng(seed)
    cams = []
    for (w, h) in sizes:
        v = rng.standard_normal(3)
        v = radius * v / np.linalg.norm(v)
        cams.append(look_at_camera(w, h, v))
    if lights:
        for c in cams:
            u = rng.standard_normal(3)
            c.light = (4.0 * u / np.linalg.norm(u)).astype(np.float32)
    return cams


def make_scene(cfg: SceneConfig, seed: int = SCENE_SEED, n_prims: Optional[int] = None) -> dict:
    """Draw the primitive parameters of a configuration.  Returns float32
    arrays; shapes: centers (P,3), scales (P,3), quats (P,4) wxyz,
    w1 (P,N,3), b1 (P,N), w2 (P,N), b2 (P,), colors (P,3) or None,
    cmlp (P,K) or None, xi (P,8) or None."""
    P = cfg.n_prims if n_prims is None else n_prims
    N = cfg.n_hidden
    rng = np.random.default_rng(seed)
    if cfg.center_dist == "uniform":
        centers = rng.uniform(-1.0, 1.0, (P, 3))
    else:
        centers = np.clip(rng.normal(0.0, 0.6, (P, 3)), -2.0, 2.0)
    scales = np.exp(rng.uniform(math.log(cfg.scale_lo), math.log(cfg.scale_hi), (P, 3)))
    quats = rng.standard_normal((P, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    w1 = rng.uniform(-1.0 / 3.0, 1.0 / 3.0, (P, N, 3))
    b1 = rng.uniform(-math.pi, math.pi, (P, N))
    w2 = rng.uniform(0.0, 1.0 / 8.0, (P, N))
    b2 = np.zeros(P)
    colors = cmlp = xi = sh = None
    if cfg.color_mode == 0:
        colors = rng.uniform(0.0, 1.0, (P, 3))
    elif cfg.color_mode == 2:
        # 16 coefficients per channel: a constant term that keeps the colour
        # mostly inside (0, 1) and a smaller view-dependent part
        sh = np.concatenate([rng.uniform(-1.5, 1.5, (P, 1, 3)), rng.uniform(-0.3, 0.3, (P, 15, 3))], axis=1)
    else:
        layers = []
        # network inputs: view direction and xi (mode 1); plus the light
        # direction (mode 3); entry point, ray direction and light direction
        # (mode 4, per ray, no xi)
        n_in = {1: 3 + XI_DIM, 3: 6 + XI_DIM, 4: 9}[cfg.color_mode]
        dims = [n_in] + [cfg.cmlp_width] * cfg.cmlp_depth + [3]
        for a, b in zip(dims[:-1], dims[1:]):
            bound = 1.0 / math.sqrt(a)
            layers.append(rng.uniform(-bound, bound, (P, b * a)))
            layers.append(rng.uniform(-bound, bound, (P, b)))
        cmlp = np.concatenate(layers, axis=1)
        assert cmlp.shape[1] == cmlp_param_count(cfg.cmlp_width, cfg.cmlp_depth, n_in)
        xi = rng.standard_normal((P, XI_DIM)) if cfg.color_mode != 4 else None
        if cfg.color_mode in (3, 4):
            colors = rng.uniform(0.0, 0.5, (P, 3))  # c_dc
    # opacity (used by Gaussians) is drawn last so the other arrays do not
    # depend on it
    opacity = rng.uniform(0.2, 0.9, P)
    # temporal weights (time-conditioned density), drawn after everything else
    wt = rng.uniform(-np.pi, np.pi, (P, N)) if cfg.temporal else None
    # with spherical harmonics, the time-dependent zero-order coefficient's
    # polynomial and Fourier coefficients a_1..4, b_1..4, c_1..4 per channel
    sh_t = rng.uniform(-0.3, 0.3, (P, 12, 3)) if cfg.temporal and cfg.color_mode == 2 else None
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return dict(P=P, N=N, omega0=cfg.omega0, color_mode=cfg.color_mode, primitive=cfg.primitive,
                opacity=f32(opacity), wt=f32(wt), time=float(cfg.time),
                cmlp_width=cfg.cmlp_width, cmlp_depth=cfg.cmlp_depth,
                centers=f32(centers), scales=f32(scales), quats=f32(quats),
                w1=f32(w1), b1=f32(b1), w2=f32(w2), b2=f32(b2),
                colors=f32(colors), cmlp=f32(cmlp), xi=f32(xi), sh=f32(sh), sh_t=f32(sh_t))


def subset_scene(scene: dict, idx) -> dict:
    """Primitives `idx` of a scene (e.g. the first 1000)."""
    out = dict(scene)
    for k in ("centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp", "xi", "sh", "opacity", "wt",
              "sh_t"):
        if scene.get(k) is not None:
            out[k] = np.ascontiguousarray(scene[k][idx])
    out["P"] = int(out["centers"].shape[0])
    return out


def make_targets(cams: List[Camera], seed: int = TARGET_SEED) -> List[np.ndarray]:
    """One U[0,1] target image (H, W, 3) float32 per camera."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.0, 1.0, (c.height, c.width, 3)).astype(np.float32) for c in cams]


def make_workload(name: str, n_prims: Optional[int] = None, sizes=None):
    """Scene, cameras and targets of configuration `name` (optionally with
    fewer primitives or other camera sizes, for tests)."""
    cfg = CONFIGS[name]
    scene = make_scene(cfg, n_prims=n_prims)
    cams = make_cameras(cfg.cams if sizes is None else sizes, lights=cfg.color_mode in (3, 4))
    return cfg, scene, cams, make_targets(cams)


def custom_scene(P, N, omega0=10.0, color_mode=0, cmlp_width=0, cmlp_depth=0,
                 seed=SCENE_SEED, center_dist="uniform", scale_lo=0.02, scale_hi=0.2, primitive=0, temporal=False):
    """A scene with the C1-C5 distributions but free sizes."""
    cfg = SceneConfig("custom", P, N, [], color_mode, cmlp_width, cmlp_depth, omega0,
                      center_dist, scale_lo, scale_hi, primitive=primitive, temporal=temporal)
    return make_scene(cfg, seed=seed)
