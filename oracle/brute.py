"""Brute-force reference for tiny scenes (test infrastructure).

Every Gaussian that is visible in float64 (finite, in front of the near plane,
able to reach alpha >= 1/255, positive determinant) is evaluated at every pixel,
in ascending (float64 depth, index) order, with the same alpha / skip / stop
rules as the renderer.  No tiles, no radius, no sort keys: this is the plain
per-pixel definition of 3D Gaussian Splatting compositing.
"""
from __future__ import annotations

import numpy as np

from .attrs64 import attrs64


def brute_ref(scene, batch, c: int = 0, e: int = 0, bg=None):
    cam = batch.cams[c]
    at = attrs64(scene, batch, c, e)
    vis = np.nonzero(at["visible64"])[0]
    order = vis[np.lexsort((vis, at["z"][vis]))]          # by depth, then index
    H, W = cam.height, cam.width
    ys, xs = np.mgrid[0:H, 0:W]
    px = xs.reshape(-1) + 0.5
    py = ys.reshape(-1) + 0.5
    T = np.ones(px.shape)
    C = np.zeros(px.shape + (3,))
    D = np.zeros(px.shape)
    added = np.zeros(px.shape, bool)
    live = np.ones(px.shape, bool)
    for g in order:
        dx = px - at["u"][g]
        dy = py - at["v"][g]
        ca, cb, cc = at["conic"][g]
        q = ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy
        a = np.minimum(0.99, at["opacity"][g] * np.exp(-0.5 * q))
        take = live & (a >= 1.0 / 255.0)
        Tn = T * (1.0 - a)
        stop = take & (Tn < 1e-4)
        live &= ~stop
        take &= ~stop
        w = np.where(take, a * T, 0.0)
        C += w[:, None] * at["rgb"][g][None, :]
        D += w * at["z"][g]
        T = np.where(take, Tn, T)
        added |= take
    bgv = np.asarray(batch.bg if bg is None else bg, np.float64).reshape(3)
    rgb = C + T[:, None] * bgv[None, :]
    with np.errstate(all="ignore"):
        depth = np.where(added, D / (1.0 - T), 0.0)
    return rgb.reshape(H, W, 3), depth.reshape(H, W), (1.0 - T).reshape(H, W)
