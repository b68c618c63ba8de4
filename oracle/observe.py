"""Observation epilogue reference (test infrastructure).

The paper trains its vision policies with image-level domain randomisation of
brightness, contrast and exposure (Sec. "Vision-Centric Manipulation
Learning"); the renderer applies it per pixel, together with the conversion to
a compact pixel format, as it writes each image.  The paper gives no
formulas; the reading used here (also listed in the design notes):

    x = rgb * gain                  (exposure as a linear gain, 2^EV)
    x = (x - 0.5) * contrast + 0.5  (contrast about mid-grey)
    x = x + brightness
    x = clamp(x, 0, 1)
    u8  = floor(255 x + 0.5)        f16 = x rounded to the nearest half

``observe64`` is that definition in float64.  The quantisation decides an
integer, so ``observe_codes`` takes it the way the kernel does, in binary32
with each step rounded (numpy float32 does not fuse), starting from the
oracle's own colour rounded to float32.  A colour within the compositing
tolerance of a code boundary can land on either side of it; such channels are
flagged and both codes are admissible.
"""
from __future__ import annotations

import numpy as np

F = np.float32


def observe64(rgb, gain=1.0, contrast=1.0, brightness=0.0):
    """Float64 epilogue of colours ``rgb`` (..., 3), parameters broadcast."""
    x = np.asarray(rgb, np.float64) * gain
    x = (x - 0.5) * contrast + 0.5
    x = x + brightness
    return np.clip(x, 0.0, 1.0)


def observe32(rgb, gain=1.0, contrast=1.0, brightness=0.0):
    """The same steps in binary32, each rounded on its own."""
    x = np.asarray(rgb, F) * F(gain)
    x = x - F(0.5)
    x = x * F(contrast)
    x = x + F(0.5)
    x = x + F(brightness)
    return np.minimum(np.maximum(x, F(0.0)), F(1.0))


def quantise_u8(x32):
    """floor(255 x + 0.5) in binary32 (x already clamped to [0, 1])."""
    x32 = np.asarray(x32, F)
    return np.floor(x32 * F(255.0) + F(0.5)).astype(np.uint8)


def observe_codes(rgb64, gain=1.0, contrast=1.0, brightness=0.0, fmt="u8", tol=1e-4):
    """Admissible observation values of oracle colours ``rgb64``.

    Returns (lo, hi): every channel's result lies in [lo, hi] (equal unless
    the channel is flagged).  A channel is flagged when moving its colour by
    ``tol`` changes the value, so that a binary32 colour that close to the
    oracle's may round to a neighbour.  ``tol`` bounds the binary32-vs-float64
    compositing difference away from threshold flips (measured at a few 1e-6;
    1e-4 keeps a wide margin while leaving most channels exact)."""
    rgb64 = np.asarray(rgb64, np.float64)
    vals = []
    for d in (-tol, 0.0, tol):
        x = observe32((rgb64 + d).astype(F), gain, contrast, brightness)
        vals.append(quantise_u8(x).astype(np.int64) if fmt == "u8" else x.astype(np.float16).astype(np.float64))
    stack = np.stack(vals)
    return stack.min(axis=0), stack.max(axis=0)
