"""Seeded synthetic workloads for the AdamW-GS step.

This module holds input generation only -- random attributes, gradients,
visibility draws and a camera rig -- and none of the optimizer's or the
visibility predicate's arithmetic.  Both the oracle-side tests and the GPU
path draw their inputs from here, so the two see identical bytes.

Shapes follow the paper's workloads: a 3DGS primitive carries a mean (3),
log-scale (3), rotation quaternion (4), opacity logit (1) and degree-3 SH
colour (48), 59 FP32 values in total (Sec. "Preliminary" of the appendix);
scenes of 0.1-6 M primitives (the Mip-NeRF360 tables).  The public datasets
themselves are not used: these generators stand in for them.

All randomness is numpy PCG64 keyed by explicit integer seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

# (name, dim, lr, dar_kind) -- dar_kind 0: none, 1: opacity sigmoid, 2: log-scale exp.
# Learning rates are the public 3DGS defaults (the paper keeps each pipeline's
# original settings); they scale the update but not the memory traffic.
GROUPS_59: List[Tuple[str, int, float, int]] = [
    ("means", 3, 1.6e-4, 0),
    ("scales", 3, 5e-3, 2),
    ("quats", 4, 1e-3, 0),
    ("opacity", 1, 5e-2, 1),
    ("sh", 48, 2.5e-3, 0),
]
# The same 59 values with the SH split the way 3DGS stores it (DC + rest).
GROUPS_60_SPLIT: List[Tuple[str, int, float, int]] = [
    ("means", 3, 1.6e-4, 0),
    ("scales", 3, 5e-3, 2),
    ("quats", 4, 1e-3, 0),
    ("opacity", 1, 5e-2, 1),
    ("sh_dc", 3, 2.5e-3, 0),
    ("sh_rest", 45, 1.25e-4, 0),
]

BETA1, BETA2, EPS = 0.9, 0.999, 1e-15
GRAD_STD = 1e-3


def rng(*key: int) -> np.random.Generator:
    """PCG64 generator keyed by a tuple of non-negative integers."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


# --------------------------------------------------------------------------
# camera rig
# --------------------------------------------------------------------------
@dataclass
class CameraSpec:
    view: np.ndarray          # (3, 4) float32, world -> camera [R|t]; camera looks along +z
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2
    z_far: float = float("inf")
    r_min: float = 0.0


def look_at(eye: np.ndarray, target: np.ndarray, up: np.ndarray) -> np.ndarray:
    """[R|t] with rows right, down, forward (x right, y down, z forward)."""
    f = target - eye
    f = f / np.linalg.norm(f)
    if abs(float(np.dot(f, up))) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1).astype(np.float32)


def fibonacci_sphere(n: int, radius: float) -> np.ndarray:
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    rho = np.sqrt(1.0 - z * z)
    phi = math.pi * (3.0 - math.sqrt(5.0)) * k
    return radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def camera_rig(n_cams: int = 200, radius: float = 15.0, fov_deg: float = 60.0,
               width: int = 1000, height: int = 1000, z_near: float = 0.2,
               z_far: float = 17.5) -> List[CameraSpec]:
    """Cameras on a Fibonacci sphere, each looking at the origin."""
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    eyes = fibonacci_sphere(n_cams, radius)
    up = np.array([0.0, 0.0, 1.0])
    return [CameraSpec(look_at(e, np.zeros(3), up), f, f, width / 2.0, height / 2.0,
                       width, height, z_near, z_far) for e in eyes]


def camera_order(n_cams: int, steps: int, seed: int = 0) -> np.ndarray:
    """Camera per step: a fresh seeded shuffle of the rig each epoch."""
    out = []
    epoch = 0
    while len(out) < steps:
        out.extend(rng(seed, 7, epoch).permutation(n_cams).tolist())
        epoch += 1
    return np.asarray(out[:steps], np.int64)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------
@dataclass
class Scene:
    n: int
    groups: List[Tuple[str, int, float, int]]
    params: Dict[str, np.ndarray] = field(default_factory=dict)   # float32 [n, dim]


def scene_uniform(n: int, seed: int = 0, groups=GROUPS_59, extent: float = 10.0) -> Scene:
    """Means ~ U[-extent, extent]^3, every other attribute ~ N(0, 1)."""
    s = Scene(n, list(groups))
    g = rng(seed, 1)
    for name, dim, _, _ in groups:
        if name == "means":
            s.params[name] = g.uniform(-extent, extent, size=(n, dim)).astype(np.float32)
        else:
            s.params[name] = g.standard_normal(size=(n, dim), dtype=np.float32)
    return s


def scene_clustered(n: int, seed: int = 0, groups=GROUPS_59, n_clusters: int = 64,
                    sigma: float = 1.5, extent: float = 10.0) -> Scene:
    """Means from an equal-weight mixture of isotropic Gaussians."""
    s = Scene(n, list(groups))
    g = rng(seed, 2)
    centres = g.uniform(-extent, extent, size=(n_clusters, 3))
    which = g.integers(0, n_clusters, size=n)
    for name, dim, _, _ in groups:
        if name == "means":
            s.params[name] = (centres[which] + sigma * g.standard_normal(size=(n, 3))).astype(np.float32)
        else:
            s.params[name] = g.standard_normal(size=(n, dim), dtype=np.float32)
    return s


def bernoulli_mask(n: int, p: float, seed: int, step: int) -> np.ndarray:
    return (rng(seed, 3, step).random(n) < p).astype(np.uint8)


def grads(n: int, groups, mask: Optional[np.ndarray], seed: int, step: int,
          std: float = GRAD_STD) -> Dict[str, np.ndarray]:
    """Photometric gradients ~ N(0, std) on visible rows, 0 elsewhere."""
    g = rng(seed, 4, step)
    out = {}
    for name, dim, _, _ in groups:
        a = (std * g.standard_normal(size=(n, dim))).astype(np.float32)
        if mask is not None:
            a[mask == 0] = 0.0
        out[name] = a
    return out


def batch_scene_sizes(n_scenes: int = 16, lo: float = 2e5, hi: float = 4e6,
                      seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Scene sizes log-uniform in [lo, hi] and visible ratios U[0.02, 0.60]."""
    g = rng(seed, 5)
    sizes = np.round(np.exp(g.uniform(math.log(lo), math.log(hi), size=n_scenes))).astype(np.int64)
    ratios = g.uniform(0.02, 0.60, size=n_scenes)
    return sizes, ratios
