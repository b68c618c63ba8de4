"""Reference images: float32-spec tile lists + float64 attributes + float64
compositing (test infrastructure).

``render_ref`` follows the renderer's definition end to end for one image:
bin (``spec32.bin_ref``), evaluate the continuous quantities in float64
(``attrs64.attrs64``), then composite every pixel front to back over its
tile's list (``composite.c``).  With the conservative radius of the binning
this equals compositing every Gaussian at every pixel in (depth, index) order
(checked against ``brute.brute_ref``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

from .attrs64 import attrs64
from .spec32 import Bins, bin_ref

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "composite.c")
_LIB = os.path.join(_HERE, "_composite.so")
_lib = None

# Relative distance to a threshold within which a float32 evaluation may take
# the other branch (see composite.c).  A float32 conic evaluated for a splat of
# anisotropy kappa carries a relative error of roughly kappa * 1e-7 in q, and
# transmittance accumulated over ~10^3 factors about 1e-4.
DEFAULT_MARGIN = 3e-4
DEFAULT_MAX_FLAGS = 3


def build_native(force: bool = False) -> str:
    """Compile composite.c with gcc (no fast-math, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = build_native()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_composite.argtypes = ([ctypes.c_int] * 4 + [P, P] + [P] * 9 + [ctypes.c_double, ctypes.c_int]
                                         + [P] * 8)
        lib.oracle_composite.restype = ctypes.c_int
        lib.oracle_pixel_variants.argtypes = ([ctypes.c_int] * 4 + [P, P] + [P] * 9 + [ctypes.c_double, ctypes.c_int]
                                              + [P] * 3)
        lib.oracle_pixel_variants.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def oracle_threads() -> int:
    """Threads the float64 compositing runs on (the float32 binning is one thread)."""
    return int(_load().oracle_threads())


def set_oracle_threads(n: int) -> int:
    """Team size of later float64 compositing calls; returns it."""
    return int(_load().oracle_set_threads(int(n)))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class RefImage:
    rgb: np.ndarray          # (H, W, 3) float64
    depth: np.ndarray        # (H, W)
    alpha: np.ndarray        # (H, W)
    var_rgb: np.ndarray      # (V, H, W, 3) admissible alternatives (V = 2^max_flags), [0] = rgb
    var_depth: np.ndarray    # (V, H, W)
    var_alpha: np.ndarray    # (V, H, W)
    nflag: np.ndarray        # (H, W) flagged decisions of the primary run
    unresolved: np.ndarray   # (H, W) bool: more flagged decisions than enumerated in var_*
    visited: np.ndarray      # (H, W) list entries visited up to termination
    bins: Optional[Bins] = None
    attrs: Optional[Dict[str, np.ndarray]] = None
    _args: Optional[tuple] = None   # compositing inputs, for pixel_variants

    def pixel_variants(self, x: int, y: int, max_m: int = 16):
        """Every admissible (rgb [V, 3], depth [V], alpha [V]) of pixel (x, y):
        all combinations of its flagged decisions, widened until no variant
        meets a flagged decision outside them.  Raises if that takes more than
        max_m flags."""
        lib = _load()
        ts, tiles_x, ranges, values, arrs, bg, margin = self._args
        n = 1 << max_m
        o_rgb, o_dep, o_alp = np.empty((n, 3)), np.empty(n), np.empty(n)
        k = lib.oracle_pixel_variants(int(x), int(y), int(ts), int(tiles_x), _ptr(ranges), _ptr(values),
                                      *[_ptr(a) for a in arrs], _ptr(bg), float(margin), int(max_m),
                                      _ptr(o_rgb), _ptr(o_dep), _ptr(o_alp))
        if k < 0:
            raise RuntimeError(f"pixel ({x}, {y}) has more than {max_m} flagged decisions")
        return o_rgb[:k].copy(), o_dep[:k].copy(), o_alp[:k].copy()


def composite64(bins: Bins, at: Dict[str, np.ndarray], width: int, height: int, ts: int, bg,
                margin: float = DEFAULT_MARGIN, max_flags: int = DEFAULT_MAX_FLAGS,
                variants: bool = True) -> RefImage:
    lib = _load()
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    u, v = f64(at["u"]), f64(at["v"])
    con = f64(at["conic"])
    ca, cb, cc = f64(con[:, 0]), f64(con[:, 1]), f64(con[:, 2])
    op, rgb, z = f64(at["opacity"]), f64(at["rgb"]), f64(at["z"])
    bg = f64(np.asarray(bg, np.float64).reshape(3))
    ranges = np.ascontiguousarray(bins.ranges, np.int64)
    values = np.ascontiguousarray(bins.values, np.uint32)
    H, W = int(height), int(width)
    nvar = 1 << max_flags
    out_rgb = np.empty((H, W, 3))
    out_depth = np.empty((H, W))
    out_alpha = np.empty((H, W))
    var_rgb = np.empty((nvar, H, W, 3)) if variants else None
    var_depth = np.empty((nvar, H, W)) if variants else None
    var_alpha = np.empty((nvar, H, W)) if variants else None
    nflag = np.empty((H, W), np.int32)
    visited = np.empty((H, W), np.int64)
    lib.oracle_composite(W, H, int(ts), int(bins.tiles_x), _ptr(ranges), _ptr(values), _ptr(u), _ptr(v),
                         _ptr(ca), _ptr(cb), _ptr(cc), _ptr(op), _ptr(rgb), _ptr(z), _ptr(bg),
                         float(margin), int(max_flags), _ptr(out_rgb), _ptr(out_depth), _ptr(out_alpha),
                         _ptr(var_rgb), _ptr(var_depth), _ptr(var_alpha), _ptr(nflag), _ptr(visited))
    if not variants:
        var_rgb, var_depth, var_alpha = out_rgb[None], out_depth[None], out_alpha[None]
    return RefImage(rgb=out_rgb, depth=out_depth, alpha=out_alpha, var_rgb=var_rgb, var_depth=var_depth,
                    var_alpha=var_alpha, nflag=nflag & 0xFFFF, unresolved=nflag >= 65536, visited=visited,
                    _args=(int(ts), int(bins.tiles_x), ranges, values, (u, v, ca, cb, cc, op, rgb, z), bg,
                           float(margin)))


def render_ref(scene, batch, c: int = 0, e: int = 0, ts: int = 16, bg=None, cutoff: float = 3.33,
               attrs: Dict[str, np.ndarray] | None = None, margin: float = DEFAULT_MARGIN,
               max_flags: int = DEFAULT_MAX_FLAGS, variants: bool = True) -> RefImage:
    """Reference image (c, e) of ``batch``; ``bg`` defaults to batch.bg."""
    cam = batch.cams[c]
    bins = bin_ref(scene, batch, c, e, ts, cutoff, attrs)
    at = attrs64(scene, batch, c, e, attrs)
    out = composite64(bins, at, cam.width, cam.height, ts, batch.bg if bg is None else bg,
                      margin, max_flags, variants)
    out.bins = bins
    out.attrs = at
    return out
