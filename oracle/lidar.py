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

* listed rays (pattern 2; the paper's non-repetitive scan LiDAR): ray k of
  the scan has its own azimuth and elevation (float32 values), direction as
  above, results in the order the rays are listed;
* a heightmap scanner (pattern 1) is a grid of parallel rays x(t) = o + t d
  with d = (0, 0, -1) from the points o = (x0 + (c + 0.5) dx, y0 + (r + 0.5)
  dy, 0) of the sensor plane; the same peak response along each ray, and the
  compositing order is the depth of the centre below that plane, max(0, -z)
  in binary32 (ties by index).

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


def is_grid(lid) -> bool:
    return int(getattr(lid, "pattern", 0)) == 1


def ray_origins(lid) -> np.ndarray:
    """(H, W, 3) float64 ray origins: the sensor origin, or (heightmap) the
    grid points of the sensor plane."""
    o = np.zeros((lid.height, lid.width, 3))
    if is_grid(lid):
        o[..., 0] = float(np.float32(lid.x0)) + (np.arange(lid.width)[None, :] + 0.5) * float(np.float32(lid.dx))
        o[..., 1] = float(np.float32(lid.y0)) + (np.arange(lid.height)[:, None] + 0.5) * float(np.float32(lid.dy))
    return o


def ray_directions(lid) -> np.ndarray:
    """(H, W, 3) float64 unit directions of a LiDAR grid (listed rays: in
    their listed order, row-major)."""
    if is_grid(lid):
        return np.broadcast_to(np.array([0.0, 0.0, -1.0]), (lid.height, lid.width, 3)).copy()
    if int(getattr(lid, "pattern", 0)) == 2:
        az = np.asarray(lid.ray_az, np.float32).astype(np.float64).reshape(lid.height, lid.width)
        el = np.asarray(lid.ray_el, np.float32).astype(np.float64).reshape(lid.height, lid.width)
        return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], axis=-1)
    az = float(np.float32(lid.az0)) + (np.arange(lid.width) + 0.5) * float(np.float32(lid.az_step))
    el = np.asarray(lid.elevations, np.float32).astype(np.float64)
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    return np.stack([ce * np.cos(az)[None], ce * np.sin(az)[None], np.broadcast_to(se, (lid.height, lid.width))],
                    axis=-1)


def centre_order(scene, batch, l: int, e: int, attrs=None) -> np.ndarray:
    """Gaussians in compositing order: binary32 centre distance (heightmap:
    depth below the sensor plane, max(0, -z)), then index."""
    at = attrs or {}
    means = np.asarray(at.get("means", scene.means), F)
    opac = np.asarray(at.get("opacities", scene.opacities), F)
    As, as_ = compose32(batch, scene, l, e)
    slot = scene.body_of() + 1
    with np.errstate(all="ignore"):
        t = affine32(As[slot], means, as_[slot])
        if is_grid(batch.cams[l]):
            depth = -t[:, 2]
            D = np.where(depth > F(0), depth, F(0)).astype(F)
            ok = np.isfinite(t).all(axis=1) & (opac >= F(1.0) / F(255.0))
        else:
            D = np.sqrt((t[:, 0] * t[:, 0] + t[:, 1] * t[:, 1]) + t[:, 2] * t[:, 2])
            ok = np.isfinite(D) & (D > F(0)) & (opac >= F(1.0) / F(255.0))
    idx = np.nonzero(ok)[0]
    keys = D.view(np.uint32)[idx]
    return idx[np.lexsort((idx, keys))]


def _sensor_frame(scene, batch, l, e, attrs):
    """Sensor-frame means m_s (N, 3), whitening matrices S^-1 R^T (N, 3, 3)
    and opacities, in float64 (rigid-body posing, then world -> sensor)."""
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
    return m_s, Wh, op


def _peak(d, m, W, o, org):
    """Peak response of Gaussians (centre m, whitening W, opacity o) along
    rays x(t) = org + t d: t* = argmin |W (org + t d - m)|^2 and alpha =
    min(0.99, o exp(-q(t*)/2)).  d and org are (rays, 3) for one Gaussian or
    (3,) for many."""
    if d.ndim == 2:                                       # many rays, one Gaussian
        rel = m[None] - org
        dw = d @ W.T
        mw = rel @ W.T
        tstar = np.einsum("ij,ij->i", dw, mw) / np.einsum("ij,ij->i", dw, dw)
        p = rel - tstar[:, None] * d
        pw = p @ W.T
    else:                                                 # one ray, many Gaussians
        rel = m - org[None]
        dw = np.einsum("nij,j->ni", W, d)
        mw = np.einsum("nij,nj->ni", W, rel)
        tstar = np.einsum("ni,ni->n", dw, mw) / np.einsum("ni,ni->n", dw, dw)
        p = rel - tstar[:, None] * d[None]
        pw = np.einsum("nij,nj->ni", W, p)
    q = np.einsum("ij,ij->i", pw, pw)
    return tstar, np.minimum(0.99, o * np.exp(-0.5 * q))


def lidar_ref(scene, batch, l: int = 0, e: int = 0, attrs=None, margin: float = 1e-3) -> LidarRef:
    """Range and hit of every ray of LiDAR slot ``l`` of env ``e``."""
    lid = batch.cams[l]
    m_s, Wh, op = _sensor_frame(scene, batch, l, e, attrs)
    d = ray_directions(lid).reshape(-1, 3)
    org = ray_origins(lid).reshape(-1, 3)
    n_rays = d.shape[0]
    near = float(np.float32(lid.near_range))
    T = np.ones(n_rays)
    Rg = np.zeros(n_rays)
    live = np.ones(n_rays, bool)
    flagged = np.zeros(n_rays, bool)
    order = centre_order(scene, batch, l, e, attrs)
    for g in order:
        tstar, a = _peak(d, m_s[g], Wh[g], op[g], org)
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


def _ray_run(tstar, a, near, margin, flips, max_flags):
    """One ray composited over per-Gaussian (t*, alpha) in compositing order,
    with the same flagged decisions as lidar_ref, taken in this order per
    Gaussian: in front of the near range, alpha >= 1/255, transmittance
    stop.  Flip bit k inverts the k-th flagged decision met.  Returns
    (range, hit, flagged decisions met)."""
    T, R, nflag = 1.0, 0.0, 0
    added = False

    def decide(value, is_flagged):
        nonlocal nflag
        if is_flagged:
            if nflag < max_flags and (flips >> nflag) & 1:
                value = not value
            nflag += 1
        return value

    for ts, al in zip(tstar, a):
        near_flag = abs(ts - near) < margin * max(1.0, near) and al >= ALPHA_MIN * (1 - margin)
        if not decide(ts > near, near_flag):
            continue
        if not decide(al >= ALPHA_MIN, abs(al * 255.0 - 1.0) < margin):
            continue
        Tn = T * (1.0 - al)
        if decide(Tn < T_MIN, abs(Tn / T_MIN - 1.0) < margin):
            break
        R += ts * al * T
        T = Tn
        added = True
    hit = 1.0 - T
    return (R / hit if added else 0.0), hit, nflag


def lidar_ray_variants(scene, batch, l: int, e: int, row: int, col: int, attrs=None, margin: float = 1e-3,
                       max_m: int = 12):
    """Every admissible (range, hit) of ray (row, col) of LiDAR slot ``l`` of
    env ``e``: all combinations of its flagged decisions, widened until no
    combination meets a flagged decision outside the enumerated ones
    (arrays of 2^m values; [0] is lidar_ref's result)."""
    lid = batch.cams[l]
    m_s, Wh, op = _sensor_frame(scene, batch, l, e, attrs)
    order = centre_order(scene, batch, l, e, attrs)
    d = ray_directions(lid)[row, col]
    org = ray_origins(lid)[row, col]
    with np.errstate(all="ignore"):
        tstar, a = _peak(d, m_s[order], Wh[order], op[order], org)
    # Gaussians below (1 - margin) / 255 at their peak can be neither taken nor
    # flagged: only the others are walked
    keep = a >= ALPHA_MIN * (1.0 - margin)
    tstar, a = tstar[keep], a[keep]
    near = float(np.float32(lid.near_range))
    m = _ray_run(tstar, a, near, margin, 0, 0)[2]
    while True:
        if m > max_m:
            raise RuntimeError(f"ray ({row}, {col}) has more than {max_m} flagged decisions")
        runs = [_ray_run(tstar, a, near, margin, f, m) for f in range(1 << m)]
        widest = max(r[2] for r in runs)
        if widest == m:
            return np.array([r[0] for r in runs]), np.array([r[1] for r in runs])
        m = widest
