"""Seeded synthetic scenes and cameras.

This module only draws random inputs (Gaussian parameters, cameras, target
images); it holds none of the rasterizer's arithmetic, so both the GPU path and
the CPU oracle can take their inputs from it.  All arrays are float32 and
structure-of-arrays, in the layouts of the public interface:

* ``means``        [3, N]  world-space centres
* ``log_scales``   [3, N]  per-axis log standard deviations
* ``quats``        [4, N]  rotation quaternions (w, x, y, z), not necessarily unit
* ``logits``       [N]     opacity logits (opacity = sigmoid(logit))
* ``sh``           [K*3, N] spherical-harmonic coefficients, plane k*3+ch
                   for SH index k = l*l + l + m and colour channel ch

Workload recipes (the paper's trained scenes are replaced by these):

* ``small``      10k Gaussians, 256x256, SH degree 0 (colour c ~ U(0,1)^3 stored
                 as DC = (c - 0.5) / Y00 so the rendered colour is c)
* ``clusters``   1M Gaussians in 64 isotropic clusters, 1280x720, SH degree 3
* ``aniso``      3M highly anisotropic Gaussians, 1920x1080, focal x1..x8
* ``tiny_grad``  200 Gaussians, 32x32, SH degree 3 (finite-difference checks)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    """Pinhole camera; world->camera rotation R (row-major 3x3) and t.

    x points right, y down, z forward; pixel (i, j) samples image point (i, j).
    """

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(3, dtype=np.float32))
    t: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3, dtype=np.float32))
    near: float = 0.2

    @property
    def campos(self) -> np.ndarray:
        """Camera centre in world space: -R^T t (float32)."""
        R = self.R.astype(np.float64)
        return (-(R.T @ self.t.astype(np.float64))).astype(np.float32)

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    @property
    def num_tiles(self) -> int:
        return self.tiles_x * self.tiles_y


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def pinhole(width, height, focal, R=None, t=None) -> Camera:
    return Camera(width, height, float(focal), float(focal), (width - 1) / 2.0, (height - 1) / 2.0,
                  np.eye(3, dtype=np.float32) if R is None else _f32(R),
                  np.zeros(3, dtype=np.float32) if t is None else _f32(t))


def look_at(eye, target=(0.0, 0.0, 0.0), width=640, height=360, focal=None) -> Camera:
    """Camera at `eye` looking at `target`, image y axis towards world -up
    (up = +y, or +z when the view direction is nearly parallel to y)."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 1.0, 0.0])
    if abs(fwd @ up) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])          # rows: camera axes in world space
    t = -R @ eye
    return pinhole(width, height, width if focal is None else focal, R, t)


def multiview_scene(seed: int = 5, n: int = 2_000_000, views: int = 32,
                    sizes=((640, 360), (1280, 720), (1920, 1080))):
    """The clustered generator with centres U([-1,1]^3) seen by `views`
    cameras at 5 * normalize(N(0, I3)) looking at the origin; camera j has
    resolution sizes[j % len(sizes)] and focal length = its width."""
    scene, _ = cluster_scene(seed, n, cube_centres=True)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    cams = []
    for j in range(views):
        d = rng.normal(size=3)
        w, h = sizes[j % len(sizes)]
        cams.append(look_at(5.0 * d / np.linalg.norm(d), width=w, height=h))
    return scene, cams


def small_scene(seed: int = 1, n: int = 10_000):
    """10k Gaussians, x,y ~ U(-1,1), z ~ U(2,6), log-scales N(-3, 0.5^2),
    opacity logits N(0,1), SH degree 0 from RGB U(0,1); 256x256, f = 256."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    log_scales = rng.normal(-3.0, 0.5, (3, n))
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    sh = (rgb - 0.5) / Y00
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 0)
    return scene, pinhole(256, 256, 256.0)


def cluster_scene(seed: int = 2, n: int = 1_000_000, clusters: int = 64, sigma: float = 0.1,
                  width: int = 1280, height: int = 720, sh_degree: int = 3, cube_centres=False):
    """Mixture of isotropic clusters (centres U([-1,1]^2 x [2,6]), members
    centre + N(0, sigma^2 I)); log-scales N(-4, 1); logits N(0, 1.5^2); SH
    coefficients N(0, 0.2^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if cube_centres:
        centres = rng.uniform(-1, 1, (3, clusters))
    else:
        centres = np.stack([rng.uniform(-1, 1, clusters), rng.uniform(-1, 1, clusters),
                            rng.uniform(2, 6, clusters)])
    member = rng.integers(0, clusters, n)
    means = centres[:, member] + rng.normal(0.0, sigma, (3, n))
    log_scales = rng.normal(-4.0, 1.0, (3, n))
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.5, n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, (3 * k, n))
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), sh_degree)
    return scene, pinhole(width, height, float(width))


def aniso_scene(seed: int = 3, n: int = 3_000_000):
    """Anisotropic Gaussians: means U([-1,1]^2 x [2,6]); base log-scale
    b ~ N(-5, 0.5^2); major/minor ratio r log-uniform in [1, 100];
    log-scales (b + ln(r)/2, b - ln(r)/2, b - ln(r)/2); random rotations;
    logits N(0,1); SH degree 3, N(0, 0.2^2).  Cameras: 1920x1080 at focal
    1920*k for k = 1..8 (a zoom-in sweep)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    b = rng.normal(-5.0, 0.5, n)
    half = 0.5 * rng.uniform(0.0, math.log(100.0), n)
    log_scales = np.stack([b + half, b - half, b - half])
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    sh = rng.normal(0.0, 0.2, (48, n))
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 3)
    cams = [pinhole(1920, 1080, 1920.0 * k) for k in range(1, 9)]
    return scene, cams


def tiny_grad_scene(seed: int = 40, n: int = 200):
    """200 Gaussians for finite differences: x,y ~ U(-0.5,0.5), z ~ U(2,4),
    log-scales N(-1.5, 0.3^2), logits N(-1, 0.5^2), SH degree 3 N(0, 0.2^2);
    32x32 image at f = 32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(2, 4, n)])
    log_scales = rng.normal(-1.5, 0.3, (3, n))
    quats = _quats(rng, n)
    logits = rng.normal(-1.0, 0.5, n)
    sh = rng.normal(0.0, 0.2, (48, n))
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 3)
    return scene, pinhole(32, 32, 32.0)


def random_scene(seed: int, n: int, width: int, height: int, focal: float, sh_degree: int = 3,
                 log_scale_mu: float = -3.0, log_scale_sd: float = 1.0, spread: float = 1.0,
                 z_range=(2.0, 6.0)):
    """Generic uniform scene for edge-case and ragged-size tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                      rng.uniform(z_range[0], z_range[1], n)])
    log_scales = rng.normal(log_scale_mu, log_scale_sd, (3, n))
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.5, n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, (3 * k, n))
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), sh_degree)
    return scene, pinhole(width, height, focal)


def target_image(seed: int, width: int, height: int) -> np.ndarray:
    """Target image U(0,1) of shape [3, H, W] for the L1 loss."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _f32(rng.uniform(0.0, 1.0, (3, height, width)))
