"""Seeded synthetic Gaussian scenes and pinhole cameras.

This module only draws inputs: random numbers, array layout and camera
poses.  It holds none of the rendering arithmetic (no projection, no colour,
no culling), so that both the fp64 CPU oracle and the GPU library can be fed
from it without sharing code with each other.

Array layout (fp32, structure of arrays, N Gaussians):

  means        [3][N]      world-space centre X
  log_scales   [3][N]      per-axis log of the scaling vector
  quats        [4][N]      rotation quaternion (w, x, y, z), not normalised
  opacity_logits [N]       peak opacity sigma = sigmoid(logit)
  sh           [3*K][N]    SH coefficients, row k*3 + c = coefficient k of
                           colour channel c, K = (degree + 1)^2

The Gaussian parameterisation (centre, rotation quaternion, scaling vector,
peak opacity, SH coefficients) is the one of the paper's background section
(Sec. 2.1).  The distributions are those of the five benchmark workloads of
this project (C1..C5); they stand in for the paper's trained PLY scenes
(Sec. 4.1), which are not available.

Camera convention (OpenCV): x right, y down, z forward.  A camera maps a
world point X to camera space p = R X + t; the world-space centre is C.  The
pixel (i, j) has its centre at (i + 0.5, j + 0.5).
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
from typing import List, Sequence

import numpy as np

__all__ = [
    "Camera", "Scene", "look_at", "c1", "c2", "c3", "c4", "c5", "c5_targets_scene",
    "fd_scene", "random_scene", "perturb", "shape_scene", "orbit_cameras",
    "sha256_arrays", "CONFIG_SEEDS",
]

CONFIG_SEEDS = {"C1": 0, "C2": 1, "C3": 2, "C4": 3, "C5": 4}


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float32, world -> camera rotation, row-major
    t: np.ndarray  # (3,) float32
    C: np.ndarray  # (3,) float32, world-space camera centre

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        self.C = np.ascontiguousarray(self.C, dtype=np.float32).reshape(3)
        # fp32 copies of the intrinsics: both consumers read these exact values
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_coeffs(self) -> int:
        return (self.sh_degree + 1) ** 2

    def arrays(self):
        return dict(means=self.means, log_scales=self.log_scales, quats=self.quats,
                    opacity_logits=self.opacity_logits, sh=self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(*(np.ascontiguousarray(a[..., idx]) for a in
                       (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)),
                     sh_degree=self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                     self.opacity_logits.copy(), self.sh.copy(), self.sh_degree)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def focal_for_hfov(width: int, hfov_deg: float = 60.0) -> float:
    """Focal length in pixels for a horizontal field of view (square pixels)."""
    return (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)


def look_at(centre, target, width, height, hfov_deg=60.0, up=(0.0, -1.0, 0.0)) -> Camera:
    """Pinhole camera at `centre` looking at `target`; `up` is world up (-y, since y points down)."""
    c = np.asarray(centre, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])  # rows: camera axes in world coordinates
    t = -R @ c
    fx = focal_for_hfov(width, hfov_deg)
    return Camera(width, height, fx, fx, width / 2.0, height / 2.0, R, t, c)


def _normalised_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return _f32(q)


def random_scene(n, seed, *, mean_lo=-1.0, mean_hi=1.0, log_scale_mu=-3.5, log_scale_sd=0.5,
                 logit_mu=0.0, logit_sd=1.5, sh_degree=0, dc_sd=0.3, rest_sd=0.3) -> Scene:
    """Uniform box scene (workload C1 shape; also the FD scene and tiny tests)."""
    rng = np.random.default_rng(seed)
    means = _f32(rng.uniform(mean_lo, mean_hi, size=(3, n)))
    log_scales = _f32(rng.normal(log_scale_mu, log_scale_sd, size=(3, n)))
    quats = _normalised_quats(rng, n)
    logits = _f32(rng.normal(logit_mu, logit_sd, size=n))
    k = (sh_degree + 1) ** 2
    dc = rng.normal(0.0, dc_sd, size=(3, n))
    rest = rng.normal(0.0, rest_sd, size=(3 * (k - 1), n))
    sh = _f32(np.concatenate([dc, rest], axis=0))
    return Scene(means, log_scales, quats, logits, sh, sh_degree)


def c1() -> tuple:
    """C1: 10,000 Gaussians in [-1,1]^3, SH degree 0, 256x256, camera at distance 3."""
    scene = random_scene(10_000, CONFIG_SEEDS["C1"], sh_degree=0, dc_sd=0.3)
    cam = Camera(256, 256, focal_for_hfov(256), focal_for_hfov(256), 128.0, 128.0,
                 np.eye(3), np.array([0.0, 0.0, 3.0]), np.array([0.0, 0.0, -3.0]))
    return scene, cam


def _shape_layout(rng, n_shapes=20):
    """10 spheres then 10 square planar patches inside the box [-5,5]^3."""
    centres = rng.uniform(-4.0, 4.0, size=(n_shapes, 3))
    radii = rng.uniform(0.5, 2.0, size=n_shapes)
    normals = rng.standard_normal((n_shapes, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    sides = rng.uniform(2.0, 6.0, size=n_shapes)
    kinds = np.array(["sphere"] * (n_shapes // 2) + ["plane"] * (n_shapes - n_shapes // 2))
    return dict(centres=centres, radii=radii, normals=normals, sides=sides, kinds=kinds)


def _plane_basis(nrm):
    helper = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(nrm, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(nrm, e1)
    return e1, e2


def shape_scene(n, seed, *, sh_degree=3, n_shapes=20, jitter=0.01, n_camera_candidates=1):
    """C2/C3 generator: points on 20 random spheres and planes, bimodal opacity, SH degree 3.

    Returns (scene, layout, candidates) where candidates is a list of
    (camera_centre, target) pairs drawn after the Gaussian arrays.
    """
    rng = np.random.default_rng(seed)
    layout = _shape_layout(rng, n_shapes)
    counts = np.full(n_shapes, n // n_shapes)
    counts[: n % n_shapes] += 1
    means = np.empty((3, n), dtype=np.float32)
    pos = 0
    for s in range(n_shapes):
        m = int(counts[s])
        c = layout["centres"][s]
        if layout["kinds"][s] == "sphere":
            d = rng.standard_normal((m, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts = c + layout["radii"][s] * d
        else:
            e1, e2 = _plane_basis(layout["normals"][s])
            h = layout["sides"][s] / 2.0
            ab = rng.uniform(-h, h, size=(m, 2))
            pts = c + ab[:, :1] * e1 + ab[:, 1:] * e2
        pts = pts + rng.normal(0.0, jitter, size=(m, 3))
        means[:, pos:pos + m] = pts.T
        pos += m
    log_scales = rng.standard_normal((3, n), dtype=np.float32) * np.float32(0.5) - np.float32(3.5)
    q = rng.standard_normal((4, n), dtype=np.float32)
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    low = rng.random(n) < 0.4
    logits = np.where(low, rng.normal(-5.0, 1.0, size=n), rng.normal(3.0, 1.0, size=n))
    k = (sh_degree + 1) ** 2
    sh = np.empty((3 * k, n), dtype=np.float32)
    sh[:3] = rng.standard_normal((3, n), dtype=np.float32) * np.float32(0.5)
    if k > 1:
        sh[3:] = rng.standard_normal((3 * (k - 1), n), dtype=np.float32) * np.float32(0.2)
    scene = Scene(_f32(means), _f32(log_scales), _f32(q), _f32(logits), sh, sh_degree)
    candidates = []
    for _ in range(n_camera_candidates):
        centre = rng.uniform(-3.0, 3.0, size=3)
        target = layout["centres"][int(rng.integers(0, n_shapes))]
        candidates.append((centre, target))
    return scene, layout, candidates


def c2(n=1_000_000):
    """C2: 1M Gaussians on spheres/planes, SH degree 3, one 1920x1080 camera inside the box."""
    scene, _, cands = shape_scene(n, CONFIG_SEEDS["C2"], n_camera_candidates=1)
    centre, target = cands[0]
    return scene, look_at(centre, target, 1920, 1080)


_C3_CAMERA_FILE = os.path.join(os.path.dirname(__file__), "c3_camera.json")


def c3(n=6_000_000, candidate=None):
    """C3: 6M Gaussians, same generator, 3840x2160.

    The camera is candidate `candidate` of the seeded candidate list; the
    default index is the recorded one (the first candidate whose pair count
    lies in [40M, 60M]), read from c3_camera.json.
    """
    if candidate is None:
        with open(_C3_CAMERA_FILE) as f:
            candidate = int(json.load(f)["candidate"])
    scene, _, cands = shape_scene(n, CONFIG_SEEDS["C3"], n_camera_candidates=candidate + 1)
    centre, target = cands[candidate]
    return scene, look_at(centre, target, 3840, 2160)


def c3_candidates(n=6_000_000, count=16):
    scene, _, cands = shape_scene(n, CONFIG_SEEDS["C3"], n_camera_candidates=count)
    return scene, [look_at(c, t, 3840, 2160) for c, t in cands]


def orbit_cameras(rng, n_views, resolutions, radius=3.0, max_elev_deg=20.0):
    """Cameras on a random orbit about the origin, looking at the origin."""
    cams = []
    for v in range(n_views):
        w, h = resolutions[v]
        az = 2.0 * math.pi * v / n_views + rng.uniform(-math.pi / n_views, math.pi / n_views)
        el = math.radians(rng.uniform(-max_elev_deg, max_elev_deg))
        centre = np.array([radius * math.cos(el) * math.sin(az), -radius * math.sin(el),
                           -radius * math.cos(el) * math.cos(az)])
        cams.append(look_at(centre, np.zeros(3), w, h))
    return cams


C4_RESOLUTIONS = [(512, 512), (1280, 720), (1920, 1080)]


def c4(n=1_000_000, n_views=64):
    """C4: C2's arrays seen by 64 orbit views of uneven resolution."""
    scene, _ = c2(n)
    rng = np.random.default_rng(CONFIG_SEEDS["C4"])
    res = [C4_RESOLUTIONS[int(i)] for i in rng.integers(0, 3, size=n_views)]
    return scene, orbit_cameras(rng, n_views, res)


def perturb(scene: Scene, seed: int, mean_sd=0.01, log_scale_sd=0.05, quat_sd=0.05,
            logit_sd=0.25, sh_sd=0.05) -> Scene:
    rng = np.random.default_rng(seed)
    out = scene.copy()
    out.means = _f32(scene.means + rng.normal(0.0, mean_sd, size=scene.means.shape))
    out.log_scales = _f32(scene.log_scales + rng.normal(0.0, log_scale_sd, size=scene.log_scales.shape))
    q = scene.quats + rng.normal(0.0, quat_sd, size=scene.quats.shape)
    out.quats = _f32(q / np.linalg.norm(q, axis=0, keepdims=True))
    out.opacity_logits = _f32(scene.opacity_logits + rng.normal(0.0, logit_sd, size=scene.opacity_logits.shape))
    out.sh = _f32(scene.sh + rng.normal(0.0, sh_sd, size=scene.sh.shape))
    return out


def c5(n=1_000_000, n_views=8, width=1920, height=1080):
    """C5: C2's arrays as parameters, 8 orbit views at 1080p, plus the perturbed target scene."""
    scene, _ = c2(n)
    rng = np.random.default_rng(CONFIG_SEEDS["C5"])
    cams = orbit_cameras(rng, n_views, [(width, height)] * n_views)
    target_scene = perturb(scene, CONFIG_SEEDS["C5"] + 1000)
    return scene, cams, target_scene


def c5_targets_scene(scene: Scene) -> Scene:
    return perturb(scene, CONFIG_SEEDS["C5"] + 1000)


def fd_scene(n=64, seed=5, width=64, height=64):
    """Finite-difference scene: 64 Gaussians in [-1,1]^3, log-scale ~ N(-2, 0.3), SH degree 3, 64x64."""
    scene = random_scene(n, seed, log_scale_mu=-2.0, log_scale_sd=0.3, sh_degree=3, dc_sd=0.5, rest_sd=0.2)
    f = focal_for_hfov(width)
    cam = Camera(width, height, f, f, width / 2.0, height / 2.0, np.eye(3), np.array([0.0, 0.0, 3.0]),
                 np.array([0.0, 0.0, -3.0]))
    return scene, cam


def sha256_arrays(arrays: Sequence[np.ndarray]) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
