"""Seeded synthetic inputs: Gaussian scenes, pinhole cameras, render requests.

This module only draws inputs.  It holds none of the renderer's arithmetic
(no projection, no covariance, no spherical-harmonics evaluation, no
compositing), so both the FP64 CPU reference and the GPU library consume the
same arrays without sharing any of the method's code.

The paper evaluates trained scenes (its Table of evaluated workloads) that are
not available here; these generators stand in for them with the shapes and
value distributions listed below (`ply.load_ply` reads trained scenes into the
same arrays).  Scene arrays (host, numpy):

    mean       float32 (3, n)            world-space centre
    log_scale  float32 (3, n)            per-axis log standard deviation
    quat       float32 (4, n)            rotation quaternion (w, x, y, z), unit norm
    opacity    float32 (n,)              in (0, 1)
    sh         float32 ((deg+1)^2, 3, n) spherical-harmonics coefficients,
                                         basis index l*l + l + m, channel-major
                                         (the device copy holds each Gaussian's
                                         coefficients contiguously)

Cameras map world to camera coordinates with x right, y down, z forward.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# DC basis value of the real orthonormal spherical harmonics, 1 / (2 sqrt(pi)).
# Used only to turn a target RGB into a degree-0 coefficient for the small
# camera-space workload (the colour the renderer should reproduce is then the
# drawn RGB itself).
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[:, idx].copy(), self.log_scale[:, idx].copy(),
                     self.quat[:, idx].copy(), self.opacity[idx].copy(),
                     self.sh[:, :, idx].copy(), self.sh_degree)

    def nbytes(self) -> int:
        return sum(a.nbytes for a in (self.mean, self.log_scale, self.quat,
                                      self.opacity, self.sh))


@dataclasses.dataclass
class Camera:
    R: np.ndarray          # (3, 3) float32, world -> camera rotation, row-major
    t: np.ndarray          # (3,) float32, world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    def packed(self) -> np.ndarray:
        """R (9), t (3), fx, fy, cx, cy, znear as float32 (the library's field order)."""
        return np.concatenate([self.R.reshape(-1), self.t,
                               np.array([self.fx, self.fy, self.cx, self.cy, self.znear])]
                              ).astype(np.float32)


def _f32(x) -> float:
    return float(np.float32(x))


def pinhole(width: int, height: int, fov_x_deg: float = 60.0, znear: float = 0.2,
            R=None, t=None) -> Camera:
    """Square-pixel pinhole with principal point at the image centre."""
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    t = np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32)
    return Camera(R, t, _f32(fx), _f32(fx), _f32(width / 2.0), _f32(height / 2.0),
                  int(width), int(height), _f32(znear))


def look_at(position, width: int, height: int, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0),
            fov_x_deg: float = 60.0, znear: float = 0.2) -> Camera:
    """Camera at `position` looking at `target` (x right, y down, z forward)."""
    p = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - p
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ p)).astype(np.float32)
    return pinhole(width, height, fov_x_deg, znear, R, t)


def sphere_position(rng: np.random.Generator, radius: float = 4.0, max_abs_cos: float = 0.9):
    """Uniform point on the sphere band |cos(theta)| <= max_abs_cos (theta from +z)."""
    z = rng.uniform(-max_abs_cos, max_abs_cos)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    s = math.sqrt(1.0 - z * z)
    return np.array([radius * s * math.cos(phi), radius * s * math.sin(phi), radius * z])


def random_pose(rng: np.random.Generator, width: int, height: int, radius: float = 4.0) -> Camera:
    return look_at(sphere_position(rng, radius), width, height)


def orbit(count: int, width: int, height: int, seed: int, radius: float = 4.0) -> list:
    """`count` poses on a horizontal circle of the radius-4 sphere band, start drawn from `seed`."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-0.9, 0.9)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    s = math.sqrt(1.0 - z * z)
    cams = []
    for k in range(count):
        phi = phi0 + 2.0 * math.pi * k / count
        cams.append(look_at([radius * s * math.cos(phi), radius * s * math.sin(phi), radius * z],
                            width, height))
    return cams


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def camera_box_scene(n: int, seed: int, log_scale_mu=math.log(0.02), log_scale_sigma=0.5) -> Scene:
    """Small camera-space workload: means U[-1,1]^2 x U[2,6], SH degree 0 from RGB ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, (3, n))
    quat = _unit_quats(rng, n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, n))
    rgb = rng.uniform(0.0, 1.0, (3, n))
    sh = ((rgb - 0.5) / _Y00)[None]
    return Scene(mean.astype(np.float32), log_scale.astype(np.float32), quat,
                 opacity.astype(np.float32), sh.astype(np.float32), 0)


def clustered_scene(n: int, seed: int, clusters: int = 64, log_scale_mu=math.log(0.01),
                    log_scale_sigma=0.7, opacity_mu=0.0, opacity_sigma=1.5, sh_degree: int = 3,
                    half_box: float = 5.0) -> Scene:
    """World-space mixture: `clusters` isotropic components, centres U[-5,5]^3, sigma U[0.25,1],
    equal weights, samples clipped to the box; SH DC ~ U[0,1], higher coefficients ~ N(0, 0.2^2)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-half_box, half_box, (clusters, 3))
    sig = rng.uniform(0.25, 1.0, clusters)
    comp = rng.integers(0, clusters, n)
    mean = centres[comp].T + sig[comp][None, :] * rng.standard_normal((3, n))
    np.clip(mean, -half_box, half_box, out=mean)
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, (3, n))
    quat = _unit_quats(rng, n)
    opacity = _sigmoid(rng.normal(opacity_mu, opacity_sigma, n))
    nb = (sh_degree + 1) ** 2
    sh = np.empty((nb, 3, n), np.float32)
    sh[0] = rng.uniform(0.0, 1.0, (3, n))
    if nb > 1:
        sh[1:] = rng.normal(0.0, 0.2, (nb - 1, 3, n))
    return Scene(mean.astype(np.float32), log_scale.astype(np.float32), quat,
                 opacity.astype(np.float32), sh, sh_degree)


# ---------------------------------------------------------------------------
# The workloads.  Each returns (scene, camera) or (scene, [cameras]).
# ---------------------------------------------------------------------------

def small_camera_space(seed: int = 1, n: int = 4096, size: int = 128):
    """4,096 Gaussians in camera space, 128x128, 60 degree FOV, SH degree 0."""
    return camera_box_scene(n, seed), pinhole(size, size, 60.0, 0.2)


def clustered_1m(seed: int = 2, n: int = 1_000_000, width: int = 1920, height: int = 1080):
    """1M Gaussians, 64 clusters, SH degree 3, camera on the radius-4 sphere, 1920x1080."""
    scene = clustered_scene(n, seed, clusters=64)
    cam = random_pose(np.random.default_rng(seed + 1000), width, height)
    return scene, cam


def clustered_3m(seed: int = 3, n: int = 3_000_000, width: int = 1920, height: int = 1080):
    """3M Gaussians, 256 clusters, same distributions as the 1M workload."""
    scene = clustered_scene(n, seed, clusters=256)
    cam = random_pose(np.random.default_rng(seed + 1000), width, height)
    return scene, cam


def dense_6m(seed: int = 5, n: int = 6_000_000, width: int = 1920, height: int = 1080):
    """Dense high-overlap stress: 6M Gaussians, log-scale N(ln 0.05, 0.5), opacity sigmoid(N(-1,1))."""
    scene = clustered_scene(n, seed, clusters=64, log_scale_mu=math.log(0.05), log_scale_sigma=0.5,
                            opacity_mu=-1.0, opacity_sigma=1.0)
    cam = random_pose(np.random.default_rng(seed + 1000), width, height)
    return scene, cam


SERVE_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (2560, 1440))


def serving_scenes(count: int = 8, n_min: int = 500_000, n_max: int = 3_000_000, seed0: int = 40,
                   scale: float = 1.0):
    """Resident scenes for the serving workload: N = linspace(0.5M, 3M, 8), seeds 40..47.
    `scale` shrinks every N (tests use it; the serving benchmark uses 1.0)."""
    ns = np.linspace(n_min, n_max, count)
    return [clustered_scene(max(1, int(round(k * scale))), seed0 + i, clusters=64)
            for i, k in enumerate(ns)]


@dataclasses.dataclass
class Request:
    rid: int
    scene: int
    width: int
    height: int
    position: np.ndarray
    arrival: float      # seconds from the start of the run (open-loop schedule)


def serving_requests(count: int, rate_hz: float, n_scenes: int = 8, seed: int = 49,
                     resolutions=SERVE_RESOLUTIONS):
    """Open-loop Poisson arrivals at `rate_hz`; scene uniform; resolution uniform; pose on the sphere."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append(Request(i, int(rng.integers(0, n_scenes)), w, h, sphere_position(rng),
                           float(arrivals[i])))
    return out


def random_keys(n: int, seed: int, hi_bits: int = 13, dup_fraction: float = 0.1):
    """Sort-test keys shaped like (bin << 32 | float bits of a positive depth), with exact duplicates."""
    rng = np.random.default_rng(seed)
    bins = rng.integers(0, 1 << hi_bits, n, dtype=np.uint64)
    depth = rng.uniform(0.2, 12.0, n).astype(np.float32).view(np.uint32).astype(np.uint64)
    keys = (bins << np.uint64(32)) | depth
    nd = int(n * dup_fraction)
    if nd and n > 1:
        src = rng.integers(0, n, nd)
        dst = rng.integers(0, n, nd)
        keys[dst] = keys[src]
    vals = rng.permutation(n).astype(np.uint32)
    return keys, vals
