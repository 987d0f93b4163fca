"""Seeded synthetic inputs: Gaussian scenes and pinhole cameras.

This module only draws random numbers and builds camera poses.  It holds none
of the rasterizer's arithmetic, so both the HIP path and the FP64 checker can
be fed from it without sharing any of the method.

The paper trains on posed photographs of real scenes with 1-5M Gaussians at
1-1.6 MP per view (Sec. 5, Tab. 1-2).  Those datasets are not available, so
every workload here is a seeded stand-in with the same orders of magnitude.

Conventions
-----------
* All arrays are float32, C-contiguous.  A scene is a dict with
  ``means [N,3]``, ``log_scales [N,3]``, ``quats [N,4]`` (w,x,y,z, not
  normalised), ``opacity_logits [N]`` and ``sh [N,16,3]`` (degree 3; row k is
  the k-th basis function, columns are RGB).
* A camera maps world to camera space as ``x_cam = R @ x_world + t`` with
  OpenCV axes (x right, y down, z forward).  Pixel (px, py) has its centre at
  (px + 0.5, py + 0.5); the principal point defaults to (W/2, H/2).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

__all__ = [
    "Camera", "make_scene", "look_at", "orbit_cameras", "fibonacci_cameras",
    "downscale", "small_scene", "paper_scale_scene", "hidden_scene", "mixed_resolution_views",
    "large_scene_views", "random_upstream", "uniform_target", "subset",
]


@dataclass
class Camera:
    R: np.ndarray            # [3,3] float32, world -> camera rotation (row-major)
    t: np.ndarray            # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    @property
    def position(self) -> np.ndarray:
        """Camera centre in world space (float64), -R^T t."""
        R = self.R.astype(np.float64)
        return -R.T @ self.t.astype(np.float64)

    def key(self):
        return (self.width, self.height)


def make_scene(n: int, seed: int, mean_range: float = 1.0, ls_mu: float = -3.5,
               ls_sigma: float = 0.3, dc_mu: float = 0.5, dc_sigma: float = 0.2,
               rest_sigma: float = 0.05) -> dict:
    """Draw a Gaussian scene as described for the synthetic workloads.

    means ~ U[-mean_range, mean_range]^3, log-scales ~ N(ls_mu, ls_sigma) per
    axis, quaternions = normalised N(0,1)^4, opacity logits ~ N(0,1), SH DC ~
    N(dc_mu, dc_sigma), higher SH bands ~ N(0, rest_sigma).  Draws are FP64
    and cast to FP32 once.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(-mean_range, mean_range, size=(n, 3))
    log_scales = rng.normal(ls_mu, ls_sigma, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.maximum(np.linalg.norm(q, axis=1, keepdims=True), 1e-12)
    logits = rng.normal(0.0, 1.0, size=(n,))
    sh = np.empty((n, 16, 3))
    sh[:, 0, :] = rng.normal(dc_mu, dc_sigma, size=(n, 3))
    sh[:, 1:, :] = rng.normal(0.0, rest_sigma, size=(n, 15, 3))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(means=f(means), log_scales=f(log_scales), quats=f(q),
                opacity_logits=f(logits), sh=f(sh))


def subset(scene: dict, idx) -> dict:
    return {k: np.ascontiguousarray(v[idx]) for k, v in scene.items()}


def look_at(position, target, width: int, height: int, fx: float, fy: float | None = None,
            near: float = 0.2, down=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at ``position`` whose +z axis points at ``target``.

    ``down`` is the world direction that should appear as image +y.
    """
    c = np.asarray(position, np.float64)
    z = np.asarray(target, np.float64) - c
    z /= np.linalg.norm(z)
    d = np.asarray(down, np.float64)
    x = np.cross(d, z)
    if np.linalg.norm(x) < 1e-9:  # looking along the down axis: pick another
        x = np.cross(np.array([0.0, 0.0, 1.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ c
    fy = fx if fy is None else fy
    return Camera(R=R.astype(np.float32), t=t.astype(np.float32), fx=float(fx), fy=float(fy),
                  cx=width / 2.0, cy=height / 2.0, width=int(width), height=int(height),
                  near=float(near))


def orbit_cameras(n_views: int, radius: float, width: int, height: int, fx: float,
                  elevation_deg: float = 0.0) -> list[Camera]:
    """Cameras on a horizontal circle around the origin; view 0 sits at (0,0,-radius)."""
    cams = []
    el = math.radians(elevation_deg)
    for k in range(n_views):
        phi = 2.0 * math.pi * k / max(n_views, 1)
        pos = (radius * math.cos(el) * math.sin(phi), -radius * math.sin(el),
               -radius * math.cos(el) * math.cos(phi))
        cams.append(look_at(pos, (0.0, 0.0, 0.0), width, height, fx))
    return cams


def fibonacci_cameras(n_views: int, radius: float, width: int, height: int, fx: float) -> list[Camera]:
    """Cameras on a Fibonacci sphere of the given radius, all looking at the origin."""
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for k in range(n_views):
        yy = 1.0 - 2.0 * (k + 0.5) / n_views
        r = math.sqrt(max(0.0, 1.0 - yy * yy))
        th = golden * k
        pos = (radius * r * math.cos(th), radius * yy, radius * r * math.sin(th))
        cams.append(look_at(pos, (0.0, 0.0, 0.0), width, height, fx))
    return cams


def downscale(cam: Camera, r: int) -> Camera:
    """The camera of a downscaled render level: W_r = floor(W/r), H_r = floor(H/r),
    focal lengths divided by r, principal point at the new image centre."""
    w, h = cam.width // r, cam.height // r
    return replace(cam, fx=cam.fx / r, fy=cam.fy / r, cx=w / 2.0, cy=h / 2.0, width=w, height=h)


# ---------------------------------------------------------------- workloads

def small_scene():
    """Small single view: 4096 Gaussians in [-1,1]^3, 128x96, fx=fy=120, camera at (0,0,-3)."""
    scene = make_scene(4096, seed=0, mean_range=1.0, ls_mu=-3.5, ls_sigma=0.3)
    cam = look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 128, 96, 120.0)
    return scene, cam


def paper_scale_scene(level: int = 1, n: int = 1_000_000, view: int = 0):
    """Paper-scale single view: 1M Gaussians in [-4,4]^3, log-scales N(-4.5,0.5),
    1600x1064, fx=fy=1400, orbit radius 6; ``level`` is the downscale factor (8/4/2/1)."""
    scene = make_scene(n, seed=0, mean_range=4.0, ls_mu=-4.5, ls_sigma=0.5)
    cam = orbit_cameras(16, 6.0, 1600, 1064, 1400.0)[view]
    return scene, downscale(cam, level)


def paper_scale_target_scene(n: int = 1_000_000):
    return make_scene(n, seed=1, mean_range=4.0, ls_mu=-4.5, ls_sigma=0.5)


def hidden_scene(n: int = 500_000, n_views: int = 64):
    """Hidden scene for the optimisation loop: 500k Gaussians drawn as the
    paper-scale scene, 64 views on a Fibonacci sphere of radius 6 at 1200x800."""
    scene = make_scene(n, seed=5, mean_range=4.0, ls_mu=-4.5, ls_sigma=0.5)
    cams = fibonacci_cameras(n_views, 6.0, 1200, 800, 1050.0)
    return scene, cams


def mixed_resolution_views():
    """16 views of the paper-scale scene: 4 each at 200x133, 400x266, 800x532, 1600x1064."""
    base = orbit_cameras(16, 6.0, 1600, 1064, 1400.0)
    cams = []
    for k, cam in enumerate(base):
        cams.append(downscale(cam, (8, 4, 2, 1)[k // 4]))
    return cams


def large_scene_views(n: int = 4_000_000):
    """Large scene: 4M Gaussians in [-20,20]^3, log-scales N(-4,0.6); 8 views at
    1920x1080 (fx=1680) and 8 at 960x540 (fx=840) on an orbit of radius 30."""
    scene = make_scene(n, seed=4, mean_range=20.0, ls_mu=-4.0, ls_sigma=0.6)
    hi = orbit_cameras(8, 30.0, 1920, 1080, 1680.0)
    lo = orbit_cameras(8, 30.0, 960, 540, 840.0, elevation_deg=20.0)
    return scene, hi + lo


def random_upstream(cam: Camera, seed: int = 3) -> np.ndarray:
    """An O(1) upstream gradient dL/dC ~ U[-1,1] of shape [3,H,W] (L = sum(w * C))."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(3, cam.height, cam.width)).astype(np.float32)


def uniform_target(cam: Camera, seed: int = 2) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(3, cam.height, cam.width)).astype(np.float32)
