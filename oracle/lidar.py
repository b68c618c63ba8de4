"""Batch LiDAR reference (test infrastructure).

The paper's simulator casts LiDAR rays against the same 3DGS scene (Sec.
"User Interface and Ecosystem Design" and its LiDAR feature table: rotating
and solid-state sensors, dynamic objects, self-occlusion).  It gives no
formulas; the reading used here (also in the design notes):

* a LiDAR is a grid of rays, beam r at elevation el[r] and column c at
  azimuth az0 + (c + 0.5) az_step, direction (cos el cos az, cos el sin az,
  sin el) in the sensor frame (x forward, y left, z up);
* a Gaussian with sensor-frame mean m, rotation R and scales S responds along
  the ray x(t) = t d with its peak: t* = argmin q(t), q(t) = |S^-1 R^T (t d -
  m)|^2, alpha = min(0.99, o exp(-q(t*)/2)), counted only if t* > near;
* Gaussians are composited front to back in the order of their centre
  distances |m| (the binary32 value, ties by index) with the image model's
  rules: skip alpha < 1/255, stop before adding when T (1 - alpha) < 1e-4;
  range = sum t* alpha T / (1 - T) (0 where nothing was added), hit = 1 - T.

``lidar_ref`` is that definition written out per ray in float64 against
every Gaussian (no binning), posing with the rigid-body kinematics of the
camera path.  Only the compositing order is taken from binary32 (the centre
distance computed like the kernel), so that both sides composite in the same
order; a ray whose threshold decision lies within ``margin`` (relative) of
its boundary is flagged.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .attrs64 import quat_to_rot64, viewmat64
from .spec32 import F, affine32, compose32

ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


@dataclass
class LidarRef:
    range: np.ndarray       # (H, W) float64
    hit: np.ndarray         # (H, W) float64
    flagged: np.ndarray     # (H, W) bool: a decision within the margin of its threshold
    order: np.ndarray       # composited Gaussians in order (indices)


def ray_directions(lid) -> np.ndarray:
    """(H, W, 3) float64 unit directions of a LiDAR grid."""
    az = float(np.float32(lid.az0)) + (np.arange(lid.width) + 0.5) * float(np.float32(lid.az_step))
    el = np.asarray(lid.elevations, np.float32).astype(np.float64)
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    return np.stack([ce * np.cos(az)[None], ce * np.sin(az)[None], np.broadcast_to(se, (lid.height, lid.width))],
                    axis=-1)


def centre_order(scene, batch, l: int, e: int, attrs=None) -> np.ndarray:
    """Gaussians in compositing order: binary32 centre distance, then index."""
    at = attrs or {}
    means = np.asarray(at.get("means", scene.means), F)
    opac = np.asarray(at.get("opacities", scene.opacities), F)
    As, as_ = compose32(batch, scene, l, e)
    slot = scene.body_of() + 1
    with np.errstate(all="ignore"):
        t = affine32(As[slot], means, as_[slot])
        D = np.sqrt((t[:, 0] * t[:, 0] + t[:, 1] * t[:, 1]) + t[:, 2] * t[:, 2])
    ok = np.isfinite(D) & (D > F(0)) & (opac >= F(1.0) / F(255.0))
    idx = np.nonzero(ok)[0]
    keys = D.view(np.uint32)[idx]
    return idx[np.lexsort((idx, keys))]


def lidar_ref(scene, batch, l: int = 0, e: int = 0, attrs=None, margin: float = 1e-3) -> LidarRef:
    """Range and hit of every ray of LiDAR slot ``l`` of env ``e``."""
    lid = batch.cams[l]
    at = attrs or {}
    mu = np.asarray(at.get("means", scene.means), np.float64)
    s = np.asarray(at.get("scales", scene.scales), np.float64)
    qg = np.asarray(at.get("quats", scene.quats), np.float64)
    op = np.asarray(at.get("opacities", scene.opacities), np.float64)
    N = mu.shape[0]
    body = scene.body_of()
    Rb = np.broadcast_to(np.eye(3), (N, 3, 3)).copy()
    tb = np.zeros((N, 3))
    if scene.n_bodies:
        pose = np.asarray(batch.poses[e], np.float64)
        Rbody = quat_to_rot64(pose[:, 0:4])
        m = body >= 0
        Rb[m] = Rbody[body[m]]
        tb[m] = pose[body[m], 4:7]
    Wv, wv = viewmat64(batch, l, e)
    m_s = (np.einsum("nij,nj->ni", Rb, mu) + tb) @ Wv.T + wv                 # sensor-frame means
    R_s = Wv[None] @ Rb @ quat_to_rot64(qg)                                   # sensor-frame rotations
    Wh = np.transpose(R_s, (0, 2, 1)) / s[:, :, None]                         # whitening S^-1 R^T

    d = ray_directions(lid).reshape(-1, 3)
    n_rays = d.shape[0]
    near = float(np.float32(lid.near_range))
    T = np.ones(n_rays)
    Rg = np.zeros(n_rays)
    live = np.ones(n_rays, bool)
    flagged = np.zeros(n_rays, bool)
    order = centre_order(scene, batch, l, e, attrs)
    for g in order:
        dw = d @ Wh[g].T                                  # (rays, 3) whitened directions
        mw = Wh[g] @ m_s[g]
        tstar = (dw @ mw) / np.einsum("ij,ij->i", dw, dw)
        p = m_s[g][None] - tstar[:, None] * d             # offset of the centre from the closest ray point
        q = np.einsum("ij,ij->i", p @ Wh[g].T, p @ Wh[g].T)
        a = np.minimum(0.99, op[g] * np.exp(-0.5 * q))
        front = tstar > near
        take = live & front & (a >= ALPHA_MIN)
        flagged |= live & front & (np.abs(a * 255.0 - 1.0) < margin)
        flagged |= live & (np.abs(tstar - near) < margin * max(1.0, near)) & (a >= ALPHA_MIN * (1 - margin))
        Tn = T * (1.0 - a)
        flagged |= take & (np.abs(Tn / T_MIN - 1.0) < margin)
        stop = take & (Tn < T_MIN)
        add = take & ~stop
        Rg = np.where(add, Rg + tstar * a * T, Rg)
        T = np.where(add, Tn, T)
        live &= ~stop
    hit = 1.0 - T
    rng = np.where(T < 1.0, Rg / np.maximum(hit, 1e-300), 0.0)
    H, W = lid.height, lid.width
    return LidarRef(range=rng.reshape(H, W), hit=hit.reshape(H, W), flagged=flagged.reshape(H, W), order=order)
