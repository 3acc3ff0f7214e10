"""Seeded synthetic inputs for the Gaussian-splatting training path.

This module only *draws inputs*: Gaussian parameter blocks, camera poses and
view orders.  It holds none of the rendering or optimisation arithmetic, so
both the GPU library and the CPU oracle can take their inputs from here
without sharing any of the method itself.

Parameter block layout (structure-of-arrays, float32, shape ``[R, N]``)::

    rows 0..2    mean mu (world x, y, z)
    rows 3..5    log-scale (per local axis)
    rows 6..9    rotation quaternion q = (w, x, y, z), not normalised
    row  10      opacity logit
    rows 11..    SH colour coefficients, coefficient-major:
                 row 11 + 3*k + channel, k = 0 .. (D+1)^2 - 1

so ``R = 11 + 3 * (D + 1)**2`` (14 for degree 0, 59 for degree 3; the paper
describes a Gaussian by 59 parameters, Section 3.1).

Priors follow the synthetic scene recipe: means uniform in the unit ball,
log-scales N(-3, 0.3^2) per axis, quaternions normalise(N(0, I4)), opacity
logits N(0, 1), diffuse RGB uniform in [0, 1] stored as the DC coefficient
(rgb - 0.5) / Y00 with Y00 = 1 / (2 sqrt(pi)), higher SH coefficients
N(0, 0.1^2).  Cameras sit on a sphere of radius 3 looking at the origin with
world up +z; the camera frame is x right, y down, z forward.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "n_rows", "sh_coeffs", "Camera", "look_at", "make_scene", "perturb_scene",
    "config_cameras", "CONFIGS", "view_order", "rng",
]

# Seeds of the recipe: scene, target perturbation, view order, MLP init, densify.
SEED_SCENE, SEED_TARGET, SEED_VIEWS, SEED_MLP, SEED_DENSIFY = 0, 1, 2, 3, 4

_Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def rng(seed: int) -> np.random.Generator:
    """Counter-based (Philox) numpy generator for a recipe seed."""
    return np.random.Generator(np.random.Philox(seed))


def sh_coeffs(degree: int) -> int:
    return (degree + 1) ** 2


def n_rows(degree: int) -> int:
    return 11 + 3 * sh_coeffs(degree)


@dataclass
class Camera:
    """Pinhole camera; pixel centres at integer coordinates."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # [3,3] world -> camera rotation (rows: right, down, forward)
    t: np.ndarray            # [3]   world -> camera translation
    campos: np.ndarray       # [3]   camera centre in world coordinates
    near: float = 0.2
    meta: dict = field(default_factory=dict)

    def world_to_cam(self) -> np.ndarray:
        """Row-major 3x4 [R | t] as float32."""
        return np.concatenate([self.R, self.t[:, None]], axis=1).astype(np.float32)


def look_at(elev_deg: float, azim_deg: float, width: int, height: int,
            radius: float = 3.0, fov_x_deg: float = 60.0) -> Camera:
    e, a = math.radians(elev_deg), math.radians(azim_deg)
    c = radius * np.array([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)])
    fwd = -c / np.linalg.norm(c)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ c
    f = float(np.float32(0.5 * width / math.tan(math.radians(fov_x_deg) / 2.0)))
    return Camera(width, height, f, f, (width - 1) / 2.0, (height - 1) / 2.0,
                  R.astype(np.float32).astype(np.float64),
                  t.astype(np.float32).astype(np.float64),
                  c.astype(np.float32).astype(np.float64),
                  meta={"elev": elev_deg, "azim": azim_deg})


def make_scene(n: int, degree: int, seed: int = SEED_SCENE) -> np.ndarray:
    """Draw an [R, n] float32 parameter block from the scene priors."""
    g = rng(seed)
    R = n_rows(degree)
    p = np.zeros((R, n), dtype=np.float64)
    d = g.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = g.random(n) ** (1.0 / 3.0)
    p[0:3] = d * r
    p[3:6] = g.normal(-3.0, 0.3, (3, n))
    q = g.standard_normal((4, n))
    p[6:10] = q / np.linalg.norm(q, axis=0, keepdims=True)
    p[10] = g.standard_normal(n)
    rgb = g.random((3, n))
    p[11:14] = (rgb - 0.5) / _Y00
    if degree > 0:
        p[14:] = g.normal(0.0, 0.1, (R - 14, n))
    return p.astype(np.float32)


def perturb_scene(p: np.ndarray, degree: int, seed: int = SEED_TARGET) -> np.ndarray:
    """Seed-perturbed copy used to render training targets."""
    g = rng(seed)
    n = p.shape[1]
    q = p.astype(np.float64).copy()
    q[0:3] += g.normal(0.0, 0.02, (3, n))
    q[3:6] += g.normal(0.0, 0.1, (3, n))
    quat = q[6:10] + g.normal(0.0, 0.1, (4, n))
    q[6:10] = quat / np.linalg.norm(quat, axis=0, keepdims=True)
    q[10] += g.normal(0.0, 0.5, n)
    rgb = q[11:14] * _Y00 + 0.5
    rgb = np.clip(rgb + g.normal(0.0, 0.1, (3, n)), 0.0, 1.0)
    q[11:14] = (rgb - 0.5) / _Y00
    if degree > 0:
        q[14:] += g.normal(0.0, 0.02, q[14:].shape)
    return q.astype(np.float32)


def _grid(elevs, azims, width, height, alt_offset=0.0):
    cams = []
    for i, e in enumerate(elevs):
        off = alt_offset if (i % 2 == 1) else 0.0
        for a in azims:
            cams.append(look_at(e, a + off, width, height))
    return cams


# Workload configurations (sizes and cameras of the five synthetic workloads).
CONFIGS = {
    "c1": dict(n=2000, degree=0, height=64, width=64, iters=100,
               elevs=[0.0], azims=[45.0 * k for k in range(8)], alt=0.0),
    "c2": dict(n=100_000, degree=3, height=480, width=640, iters=2000,
               elevs=[-30.0, -10.0, 10.0, 30.0], azims=[45.0 * k for k in range(8)], alt=22.5),
    "c3": dict(n=1_000_000, degree=3, height=1080, width=1600, iters=None,
               elevs=list(np.linspace(-60.0, 60.0, 10)), azims=[36.0 * k for k in range(10)], alt=0.0),
    "c4": dict(n=3_000_000, degree=3, height=1080, width=1920, iters=30000,
               elevs=list(np.linspace(-60.0, 60.0, 10)), azims=[24.0 * k for k in range(15)], alt=0.0),
}
CONFIGS["c5"] = dict(CONFIGS["c4"])


def config_cameras(name: str, width: int | None = None, height: int | None = None):
    c = CONFIGS[name]
    return _grid(c["elevs"], c["azims"], width or c["width"], height or c["height"], c["alt"])


def view_order(n_views: int, n_iters: int, seed: int = SEED_VIEWS) -> np.ndarray:
    """Per-epoch seeded permutations of the training views, concatenated."""
    g = rng(seed)
    out = []
    while sum(len(o) for o in out) < n_iters:
        out.append(g.permutation(n_views))
    return np.concatenate(out)[:n_iters].astype(np.int64)
