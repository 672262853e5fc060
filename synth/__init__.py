"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module only draws random numbers and builds camera poses. It holds none
of the rendering, decoding or optimisation arithmetic: both the CPU oracle and
the HIP path receive the arrays produced here and nothing else.

Scene layout (one row per Gaussian, float32, C-contiguous):
  mean          [n, 3]   world position p (Sec. 3.1, Eq. 1)
  log_scale     [n, 3]   log of the per-axis standard deviations (Sigma = R S S^T R^T)
  quat          [n, 4]   rotation as (w, x, y, z), unit norm as drawn
  opacity_logit [n]      alpha before the sigmoid
  channels      [n, C]   RGB (3) | compact semantic feature s_G (d_s) | uncertainty u (1)
                         (Sec. 3.4.1 and 3.4.2: colour, s_G and u are all blended)

Draw order for a scene (one numpy Generator seeded with `seed`):
  mean xyz, log_scale, quat, opacity_logit, rgb, semantic, uncertainty.

Cameras use world-to-camera rotation R (row-major 3x3) and translation t with
OpenCV axes (x right, y down, z forward). Pixel (i, j) has its centre at
(i + 0.5, j + 0.5); the principal point is the image centre.
"""
from __future__ import annotations

import dataclasses
import numpy as np

# Volumes used by the workload configurations.
VOL_C1 = ((-1.0, 1.0), (-1.0, 1.0), (2.0, 6.0))       # 128x128 single view
VOL_C2 = ((-4.0, 4.0), (-4.0, 4.0), (2.0, 12.0))      # 1080x720 single view
VOL_CUBE = ((-4.0, 4.0), (-4.0, 4.0), (-4.0, 4.0))    # sphere-rig scenes

RESOLUTIONS_C3 = ((640, 480), (960, 540), (1080, 720), (1280, 720), (1920, 1080))


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    channels: np.ndarray
    d_sem: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    @property
    def n_channels(self) -> int:
        return int(self.channels.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[idx].copy(), self.log_scale[idx].copy(), self.quat[idx].copy(),
                     self.opacity_logit[idx].copy(), self.channels[idx].copy(), self.d_sem)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # [3, 3] float64, world -> camera
    t: np.ndarray          # [3] float64

    def as_tuple(self):
        return (int(self.width), int(self.height), float(self.fx), float(self.fy),
                float(self.cx), float(self.cy),
                tuple(float(v) for v in np.asarray(self.R, np.float64).reshape(9)),
                tuple(float(v) for v in np.asarray(self.t, np.float64).reshape(3)))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def make_scene(n: int, seed: int, volume=VOL_C1, d_sem: int = 8,
               log_scale_mu: float = -3.0, log_scale_sigma: float = 0.5) -> Scene:
    """Draw n Gaussians: means uniform in `volume`, log-scales N(mu, sigma) per
    axis, rotations uniform (normalised 4-d normals), opacity logits N(0, 1),
    RGB U[0, 1], semantic features N(0, 1), uncertainty sigmoid(N(0, 1))."""
    rng = np.random.default_rng(seed)
    lo = np.array([v[0] for v in volume])
    hi = np.array([v[1] for v in volume])
    mean = (lo + (hi - lo) * rng.random((n, 3))).astype(np.float32)
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, (n, 3)).astype(np.float32)
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    quat = q.astype(np.float32)
    opacity_logit = rng.normal(0.0, 1.0, n).astype(np.float32)
    rgb = rng.random((n, 3))
    sem = rng.normal(0.0, 1.0, (n, d_sem))
    unc = _sigmoid(rng.normal(0.0, 1.0, (n, 1)))
    channels = np.concatenate([rgb, sem, unc], axis=1).astype(np.float32)
    return Scene(np.ascontiguousarray(mean), np.ascontiguousarray(log_scale),
                 np.ascontiguousarray(quat), np.ascontiguousarray(opacity_logit),
                 np.ascontiguousarray(channels), d_sem)


def camera_front(width: int, height: int, focal: float) -> Camera:
    """Identity pose at the origin looking down +z."""
    return Camera(width, height, float(focal), float(focal), width / 2.0, height / 2.0,
                  np.eye(3), np.zeros(3))


def look_at(position, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World-to-camera (R, t) for a camera at `position` looking at `target`,
    OpenCV axes, with `up` mapped to -y on screen (falls back to +z when the
    view direction is nearly parallel to `up`)."""
    pos = np.asarray(position, np.float64)
    z = np.asarray(target, np.float64) - pos
    z /= np.linalg.norm(z)
    upv = np.asarray(up, np.float64)
    if abs(float(np.dot(z, upv))) > 0.99:
        upv = np.array([0.0, 0.0, 1.0])
    y = -(upv - np.dot(upv, z) * z)
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    R = np.stack([x, y, z], axis=0)
    t = -R @ pos
    return R, t


def cameras_sphere(n_views: int, seed: int, radius: float = 8.0, resolutions=None,
                   focal_from_width: bool = True):
    """n_views cameras on a sphere of `radius` around the origin, looking at it.
    Positions radius * g / |g| with g ~ N(0, I3); resolutions drawn uniformly
    from `resolutions` (a single (W, H) pair or a tuple of pairs); focal = W."""
    rng = np.random.default_rng(seed)
    if resolutions is None:
        resolutions = ((1920, 1080),)
    if isinstance(resolutions[0], int):
        resolutions = (tuple(resolutions),)
    cams = []
    for _ in range(n_views):
        g = rng.normal(0.0, 1.0, 3)
        pos = radius * g / np.linalg.norm(g)
        k = int(rng.integers(0, len(resolutions)))
        w, h = resolutions[k]
        R, t = look_at(pos)
        f = float(w) if focal_from_width else float(max(w, h))
        cams.append(Camera(w, h, f, f, w / 2.0, h / 2.0, R, t))
    return cams


def upstream_grads(cams, n_channels: int, seed: int):
    """dL/d(output) per pixel and channel, N(0, 1), planar [C][H][W] per view,
    concatenated over views (float32)."""
    rng = np.random.default_rng(seed)
    total = sum(n_channels * c.height * c.width for c in cams)
    return rng.normal(0.0, 1.0, total).astype(np.float32)


def targets_l1(cams, n_channels: int, d_sem: int, seed: int):
    """Seeded L1 targets, planar [C][H][W] per view concatenated: RGB U[0, 1],
    semantic features N(0, 1), uncertainty target 0."""
    rng = np.random.default_rng(seed)
    out = []
    for c in cams:
        hw = c.height * c.width
        rgb = rng.random((3, hw))
        sem = rng.normal(0.0, 1.0, (d_sem, hw))
        unc = np.zeros((n_channels - 3 - d_sem, hw))
        out.append(np.concatenate([rgb, sem, unc], axis=0).reshape(-1))
    return np.concatenate(out).astype(np.float32)


def codebook(n_codes: int, dim: int, seed: int):
    """n_codes rows N(0, I) normalised to unit length (float32)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(0.0, 1.0, (n_codes, dim))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    return c.astype(np.float32)


def projection(dim_out: int, dim_in: int, seed: int):
    """Fixed seeded dim_in -> dim_out projection, entries N(0, 1/dim_in) (float32)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0 / np.sqrt(dim_in), (dim_out, dim_in)).astype(np.float32)


def mlp_init(sizes, seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights [out][in] and biases,
    float32, in layer order."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        k = 1.0 / np.sqrt(fi)
        ws.append(rng.uniform(-k, k, (fo, fi)).astype(np.float32))
        bs.append(rng.uniform(-k, k, fo).astype(np.float32))
    return ws, bs


# Named workloads -----------------------------------------------------------

def workload_c1(seed: int = 1):
    scene = make_scene(10_000, seed, VOL_C1, d_sem=8)
    cams = [camera_front(128, 128, 128.0)]
    return scene, cams


def workload_c2(seed: int = 2):
    scene = make_scene(300_000, seed, VOL_C2, d_sem=8)
    cams = [camera_front(1080, 720, 1080.0)]
    return scene, cams


def workload_1m_1080p(seed: int = 6):
    """1M Gaussians in the [-4, 4]^3 cube, one 1920x1080 camera on the r=8 sphere."""
    scene = make_scene(1_000_000, seed, VOL_CUBE, d_sem=8)
    cams = cameras_sphere(1, seed + 100, 8.0, (1920, 1080))
    return scene, cams


def workload_c3(seed: int = 3):
    scene = make_scene(1_000_000, seed, VOL_CUBE, d_sem=8)
    cams = cameras_sphere(16, seed + 100, 8.0, RESOLUTIONS_C3)
    return scene, cams


def workload_c4(seed: int = 4):
    scene = make_scene(1_000_000, seed, VOL_CUBE, d_sem=8)
    cams = cameras_sphere(32, seed + 100, 8.0, (1920, 1080))
    return scene, cams


def workload_c5(seed: int = 5):
    scene = make_scene(3_000_000, seed, VOL_CUBE, d_sem=16)
    cams = cameras_sphere(4, seed + 100, 8.0, (1920, 1080))
    return scene, cams
