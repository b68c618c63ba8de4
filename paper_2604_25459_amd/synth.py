"""Seeded synthetic inputs for the batched Gaussian-splatting renderer.

This module is shared by the CPU oracle and by the GPU path, so it holds none of
the rendering arithmetic: it only draws random numbers (in float64, rounded to
float32), places look-at cameras, and states pinhole intrinsics for a vertical
field of view.  Everything it returns is a plain numpy array or dataclass.

Workloads follow the paper's batch-rendering setting (Sec. "Batch Renderer
Optimization": 2048 environments at 640x480, scenes made of a static background
plus Gaussian clusters bound to rigid bodies, RLGK).  The paper's reconstructed,
pruned scenes are not available; these seeded scenes stand in for them.

Conventions
-----------
* World frame right-handed, +z up.  Cameras are OpenCV style (x right, y down,
  z forward).  A viewmat is the world->camera transform [R | t] (3x4).
* Quaternions are (w, x, y, z).  Scales are linear (log-scales are drawn and
  exponentiated here, in float64).  Opacities are activated values in (0, 1).
* Body poses are world-from-body (qw, qx, qy, qz, tx, ty, tz).
* Gaussian index g: static background first, then body 0 .. B-1, each in
  storage order; ``body_offsets`` (B+1 entries) marks the ranges.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

SEED_BASE = 260425459

# Stream identifiers for SeedSequence spawn keys: one independent stream per
# purpose, so adding draws to one never shifts another.
_S_SCENE, _S_CAMERA, _S_POSE, _S_TRACE = 0, 1, 2, 3


def sh_coeff_count(degree: int) -> int:
    """Number of SH coefficients per colour channel for a given degree."""
    return (degree + 1) ** 2


@dataclass
class Scene:
    means: np.ndarray         # (N, 3) float32; body Gaussians in their body frame
    scales: np.ndarray        # (N, 3) float32, linear, > 0
    quats: np.ndarray         # (N, 4) float32 (w, x, y, z), not normalised
    opacities: np.ndarray     # (N,)  float32 in (0, 1)
    sh: np.ndarray            # (N, K, 3) float32, K = (degree + 1)^2
    sh_degree: int
    body_offsets: np.ndarray  # (B + 1,) int64, [0, off[0]) static, body b = [off[b], off[b+1])

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_bodies(self) -> int:
        return int(self.body_offsets.shape[0]) - 1

    def body_of(self) -> np.ndarray:
        """Per-Gaussian body id, -1 for static Gaussians (int32)."""
        out = np.full(self.n, -1, dtype=np.int32)
        off = self.body_offsets
        for b in range(self.n_bodies):
            out[off[b]:off[b + 1]] = b
        return out


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near: float = 0.01
    attach_body: int = -1     # >= 0: viewmats of this slot are body -> camera offsets


@dataclass
class Batch:
    cams: List[Camera]        # C camera slots, each with its own resolution
    viewmats: np.ndarray      # (C, E, 3, 4) float32, world -> camera
    poses: np.ndarray         # (E, B, 7) float32, world-from-body
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))

    @property
    def n_envs(self) -> int:
        return int(self.viewmats.shape[1])

    @property
    def n_cams(self) -> int:
        return int(self.viewmats.shape[0])

    @property
    def n_images(self) -> int:
        return self.n_envs * self.n_cams

    def image_index(self, c: int, e: int) -> int:
        """Images are ordered camera-slot-major: i = c * E + e."""
        return c * self.n_envs + e

    def subset(self, envs: Sequence[int]) -> "Batch":
        envs = np.asarray(envs, dtype=np.int64)
        return Batch(cams=list(self.cams), viewmats=np.ascontiguousarray(self.viewmats[:, envs]),
                     poses=np.ascontiguousarray(self.poses[envs]), bg=self.bg.copy())


# --------------------------------------------------------------------------
# camera helpers (input preparation: intrinsics and look-at extrinsics)
# --------------------------------------------------------------------------

def pinhole(width: int, height: int, fov_y_deg: float, near: float = 0.01) -> Camera:
    """Square-pixel pinhole with a vertical field of view, principal point at
    the image centre.  Values computed in float64 and rounded to float32."""
    fy = (0.5 * height) / math.tan(math.radians(fov_y_deg) * 0.5)
    f32 = lambda x: float(np.float32(x))
    return Camera(width=int(width), height=int(height), fx=f32(fy), fy=f32(fy),
                  cx=f32(0.5 * width), cy=f32(0.5 * height), near=f32(near))


def look_at(eye, target) -> np.ndarray:
    """World->camera [R | t] (float64, 3x4) for an OpenCV camera at ``eye``
    looking at ``target`` with +z as up (or +y when looking nearly along z)."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    f = target - eye
    f = f / np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) <= 0.99 else np.array([0.0, 1.0, 0.0])
    x = np.cross(f, up)
    x = x / np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f], axis=0)
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1)


# --------------------------------------------------------------------------
# random draws
# --------------------------------------------------------------------------

def _rng(cfg_seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(cfg_seed, spawn_key=tuple(key))))


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _sphere_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def draw_gaussians(rng: np.random.Generator, n: int, half_box: float, log_scale_mu: float,
                   log_scale_sigma: float, sh_degree: int):
    """Draw n Gaussians: means U[-h, h]^3, log-scales N(mu, sigma) per axis,
    uniform unit quaternions, opacity = sigmoid(N(0, 1)), SH DC ~ U(0, 1) and
    higher bands ~ N(0, 0.1).  Draw order is fixed (means, log-scales, quats,
    opacity logits, SH DC, SH rest).  Returns float32 arrays."""
    K = sh_coeff_count(sh_degree)
    means = rng.uniform(-half_box, half_box, size=(n, 3))
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    quats = _unit_quats(rng, n)
    logits = rng.standard_normal(n)
    dc = rng.uniform(0.0, 1.0, size=(n, 1, 3))
    rest = rng.normal(0.0, 0.1, size=(n, K - 1, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return (f32(means), f32(np.exp(log_scales)), f32(quats),
            f32(1.0 / (1.0 + np.exp(-logits))), f32(np.concatenate([dc, rest], axis=1)))


def make_scene(seed: int, n_static: int, n_bodies: int, per_body: int, *, sh_degree: int,
               half_box: float = 1.0, body_half_box: float = 0.25,
               log_scale_mu: float = math.log(0.03), log_scale_sigma: float = 0.5,
               body_log_scale_mu: float | None = None, body_log_scale_sigma: float | None = None) -> Scene:
    """Static background (means in [-half_box, half_box]^3) plus ``n_bodies``
    clusters of ``per_body`` Gaussians with body-local means in
    [-body_half_box, body_half_box]^3 (about a half-metre object)."""
    rng = _rng(seed, _S_SCENE)
    parts = [draw_gaussians(rng, n_static, half_box, log_scale_mu, log_scale_sigma, sh_degree)]
    bmu = log_scale_mu if body_log_scale_mu is None else body_log_scale_mu
    bsig = log_scale_sigma if body_log_scale_sigma is None else body_log_scale_sigma
    for _ in range(n_bodies):
        parts.append(draw_gaussians(rng, per_body, body_half_box, bmu, bsig, sh_degree))
    cat = lambda j: np.ascontiguousarray(np.concatenate([p[j] for p in parts], axis=0))
    offsets = np.array([n_static + b * per_body for b in range(n_bodies + 1)], dtype=np.int64)
    return Scene(means=cat(0), scales=cat(1), quats=cat(2), opacities=cat(3), sh=cat(4),
                 sh_degree=sh_degree, body_offsets=offsets)


def random_poses(rng: np.random.Generator, n_envs: int, n_bodies: int, half_box: float = 1.0) -> np.ndarray:
    """Per-env world-from-body poses: uniform unit quaternion, translation U[-h, h]^3."""
    q = _unit_quats(rng, n_envs * n_bodies).reshape(n_envs, n_bodies, 4)
    t = rng.uniform(-half_box, half_box, size=(n_envs, n_bodies, 3))
    return np.ascontiguousarray(np.concatenate([q, t], axis=2), dtype=np.float32)


def orbit_viewmats(rng: np.random.Generator, n: int, r_lo: float, r_hi: float,
                   targets: np.ndarray | None = None) -> np.ndarray:
    """n look-at cameras at radius U[r_lo, r_hi] from their target (origin by
    default), direction uniform on the sphere.  Returns (n, 3, 4) float32."""
    d = _sphere_dirs(rng, n)
    r = rng.uniform(r_lo, r_hi, size=n) if r_hi > r_lo else np.full(n, r_lo)
    tg = np.zeros((n, 3)) if targets is None else np.asarray(targets, np.float64)
    out = np.empty((n, 3, 4), np.float64)
    for k in range(n):
        out[k] = look_at(tg[k] + r[k] * d[k], tg[k])
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# LiDAR grids
# --------------------------------------------------------------------------
@dataclass
class LidarSpec:
    """A ray grid (sensor frame x forward, y left, z up).  pattern 0
    (angular): ``height`` beams at ``elevations`` (radians, ascending) x
    ``width`` columns at azimuths az0 + (c + 0.5) az_step, rays from the
    sensor origin.  pattern 1 (heightmap grid): ``height`` x ``width``
    parallel rays along -z from the sensor's z = 0 plane, ray (r, c) starting
    at (x0 + (c + 0.5) dx, y0 + (r + 0.5) dy, 0).  pattern 2 (listed rays):
    ray k of the ``height`` x ``width`` rays at azimuth ray_az[k] and
    elevation ray_el[k] (arrays of that shape, row-major), from the sensor
    origin."""
    width: int
    height: int
    az0: float
    az_step: float
    elevations: np.ndarray
    near_range: float = 0.05
    attach_body: int = -1
    pattern: int = 0
    x0: float = 0.0
    y0: float = 0.0
    dx: float = 0.0
    dy: float = 0.0
    ray_az: np.ndarray = None
    ray_el: np.ndarray = None


@dataclass
class LidarBatch:
    cams: List[LidarSpec]     # L LiDAR slots (named like camera slots, so posing code is shared)
    viewmats: np.ndarray      # (L, E, 3, 4) float32 world -> sensor (body -> sensor when attached)
    poses: np.ndarray         # (E, B, 7) float32

    @property
    def n_envs(self) -> int:
        return int(self.viewmats.shape[1])


def rotating_lidar(beams: int, columns: int, el_lo_deg: float, el_hi_deg: float, near: float = 0.05) -> LidarSpec:
    """Full-turn LiDAR with evenly spaced beams (float64 angles rounded to float32)."""
    el = np.radians(np.linspace(el_lo_deg, el_hi_deg, beams)).astype(np.float32)
    return LidarSpec(width=columns, height=beams, az0=float(np.float32(-math.pi)),
                     az_step=float(np.float32(2.0 * math.pi / columns)), elevations=el,
                     near_range=float(np.float32(near)))


def sector_lidar(beams: int, columns: int, az_deg: float, el_lo_deg: float, el_hi_deg: float,
                 near: float = 0.05) -> LidarSpec:
    """Solid-state LiDAR covering azimuths [-az/2, az/2] in front of the sensor."""
    el = np.radians(np.linspace(el_lo_deg, el_hi_deg, beams)).astype(np.float32)
    a = math.radians(az_deg)
    return LidarSpec(width=columns, height=beams, az0=float(np.float32(-0.5 * a)),
                     az_step=float(np.float32(a / columns)), elevations=el, near_range=float(np.float32(near)))


def rosette_lidar(rows: int, cols: int, half_fov_deg: float = 35.0, petals: float = 5.0, s0: float = 0.0,
                  near: float = 0.05) -> LidarSpec:
    """Non-repetitive (rosette) scan of rows * cols rays: the points of the
    rose curve rho(s) = A sin(petals s), (azimuth, elevation) = rho (cos s,
    sin s), A = half_fov, at s = s0 + k ds with ds = pi (3 - sqrt 5) (the
    golden angle), so no two scans of successive s0 repeat their rays.
    Angles in float32, shape (rows, cols)."""
    n = rows * cols
    s = s0 + np.arange(n, dtype=np.float64) * (math.pi * (3.0 - math.sqrt(5.0)))
    rho = math.radians(half_fov_deg) * np.sin(petals * s)
    az = (rho * np.cos(s)).astype(np.float32).reshape(rows, cols)
    el = (rho * np.sin(s)).astype(np.float32).reshape(rows, cols)
    return LidarSpec(width=cols, height=rows, az0=0.0, az_step=0.0, elevations=np.zeros(0, np.float32),
                     near_range=float(np.float32(near)), pattern=2, ray_az=az, ray_el=el)


def height_grid(rows: int, cols: int, spacing: float, near: float = 0.05) -> LidarSpec:
    """Heightmap scanner centred on the sensor: rows x cols parallel rays along
    -z at ``spacing`` metres (float32 parameters)."""
    f = lambda v: float(np.float32(v))
    return LidarSpec(width=cols, height=rows, az0=0.0, az_step=0.0, elevations=np.zeros(0, np.float32),
                     near_range=f(near), pattern=1, x0=f(-0.5 * cols * spacing), y0=f(-0.5 * rows * spacing),
                     dx=f(spacing), dy=f(spacing))


def sensor_viewmats(rng: np.random.Generator, n: int, r_lo: float, r_hi: float, z: float = 0.0) -> np.ndarray:
    """n level sensors at radius U[r_lo, r_hi] from the z axis, height z,
    random heading.  World -> sensor [R^T | -R^T c], (n, 3, 4) float32."""
    out = np.empty((n, 3, 4), np.float64)
    ang = rng.uniform(0.0, 2.0 * math.pi, n)
    rad = rng.uniform(r_lo, r_hi, n) if r_hi > r_lo else np.full(n, r_lo)
    yaw = rng.uniform(-math.pi, math.pi, n)
    for k in range(n):
        c = np.array([rad[k] * math.cos(ang[k]), rad[k] * math.sin(ang[k]), z])
        cy, sy = math.cos(yaw[k]), math.sin(yaw[k])
        R = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])       # sensor axes in world
        out[k, :, :3] = R.T
        out[k, :, 3] = -R.T @ c
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

CONFIG_NAMES = {
    0: "plain 1x128x96, 4096 G, SH1, no bodies",
    1: "64 envs x 320x240, 100k bg + 8x5k bodies, SH3",
    2: "2048 envs x 640x480, 200k bg + 10x10k bodies, SH3",
    3: "512 envs x {128x128 wrist 90deg, 640x480 head}, 500k bg + 12x8k bodies",
    4: "serving stream, Poisson 200 req/s",
}


def config_seed(cfg: int) -> int:
    return SEED_BASE + cfg


def make_config(cfg: int, n_envs: int | None = None, step: int = 0):
    """Scene and step-``step`` batch of workload ``cfg`` (0..3).  ``n_envs``
    optionally truncates the batch to its first environments (the draws of the
    kept environments do not change)."""
    s = config_seed(cfg)
    if cfg == 0:
        scene = make_scene(s, 4096, 0, 0, sh_degree=1, half_box=1.0)
        rng = _rng(s, _S_CAMERA)
        cams = [pinhole(128, 96, 60.0)]
        vm = orbit_viewmats(rng, 1, 3.0, 3.0)
        E = 1
        poses = np.zeros((E, 0, 7), np.float32)
        batch = Batch(cams=cams, viewmats=vm[None], poses=poses)
    elif cfg == 1:
        E = 64
        scene = make_scene(s, 100_000, 8, 5_000, sh_degree=3, half_box=4.0)
        rng = _rng(s, _S_CAMERA)
        vm = orbit_viewmats(rng, E, 3.0, 6.0)
        poses = random_poses(_rng(s, _S_POSE, step), E, 8)
        batch = Batch(cams=[pinhole(320, 240, 60.0)], viewmats=vm[None], poses=poses)
    elif cfg == 2:
        E = 2048
        scene = make_scene(s, 200_000, 10, 10_000, sh_degree=3, half_box=4.0)
        rng = _rng(s, _S_CAMERA)
        vm = orbit_viewmats(rng, E, 3.0, 6.0)          # cameras fixed per env
        poses = random_poses(_rng(s, _S_POSE, step), E, 10)   # resampled each step
        batch = Batch(cams=[pinhole(640, 480, 60.0)], viewmats=vm[None], poses=poses)
    elif cfg == 3:
        E = 512
        scene = make_scene(s, 500_000, 12, 8_000, sh_degree=3, half_box=4.0,
                           log_scale_mu=math.log(0.01), log_scale_sigma=0.7,
                           body_log_scale_mu=math.log(0.03), body_log_scale_sigma=0.5)
        rng = _rng(s, _S_CAMERA)
        poses = random_poses(_rng(s, _S_POSE, step), E, 12)
        wrist_targets = poses[:, 0, 4:7].astype(np.float64)
        wrist = orbit_viewmats(rng, E, 0.3, 1.0, targets=wrist_targets)
        head = orbit_viewmats(rng, E, 3.0, 6.0)
        cams = [pinhole(128, 128, 90.0, near=0.02), pinhole(640, 480, 60.0)]
        batch = Batch(cams=cams, viewmats=np.stack([wrist, head], axis=0), poses=poses)
    else:
        raise ValueError(f"no batch workload for config {cfg}")
    if n_envs is not None and n_envs < batch.n_envs:
        batch = batch.subset(range(n_envs))
    return scene, batch


def make_poses(cfg: int, step: int, n_envs: int, n_bodies: int) -> np.ndarray:
    """Body poses of workload ``cfg`` at ``step`` (the same draws make_config
    uses for that step), without regenerating the scene."""
    return random_poses(_rng(config_seed(cfg), _S_POSE, step), n_envs, n_bodies)


# --------------------------------------------------------------------------
# serving stream (workload 4)
# --------------------------------------------------------------------------

SERVE_RESOLUTIONS = [(128, 128), (320, 240), (640, 480)]


@dataclass
class Request:
    arrival_s: float
    n_envs: int
    width: int
    height: int
    scene: int          # index into the scene pool


def serving_pool_scene(k: int) -> Scene:
    """Scene k of the 32-scene pool: log-uniform [50k, 1M] background in
    [-4, 4]^3 plus U{4..16} bodies of 5k Gaussians, SH degree 3."""
    rng = _rng(config_seed(4), _S_SCENE, k)
    n_bg = int(math.exp(rng.uniform(math.log(50_000), math.log(1_000_000))))
    n_b = int(rng.integers(4, 17))
    return make_scene(config_seed(4) * 1000 + k, n_bg, n_b, 5_000, sh_degree=3, half_box=4.0)


def serving_trace(rate_hz: float = 200.0, duration_s: float = 60.0, pool: int = 32) -> List[Request]:
    """Poisson arrivals; per request envs = floor(exp(U[0, ln 257))) in [1, 256],
    a resolution drawn uniformly, and a scene drawn uniformly from the pool."""
    rng = _rng(config_seed(4), _S_TRACE)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        e = int(math.floor(math.exp(rng.uniform(0.0, math.log(257.0)))))
        w, h = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
        out.append(Request(arrival_s=t, n_envs=max(1, min(256, e)), width=w, height=h,
                           scene=int(rng.integers(0, pool))))
    return out


def serving_batch(req: Request, scene: Scene, req_index: int) -> Batch:
    """Cameras and poses for one serving request (seeded by its index)."""
    rng = _rng(config_seed(4), _S_POSE, req_index)
    vm = orbit_viewmats(rng, req.n_envs, 3.0, 6.0)
    poses = random_poses(rng, req.n_envs, scene.n_bodies)
    return Batch(cams=[pinhole(req.width, req.height, 60.0)], viewmats=vm[None], poses=poses)
