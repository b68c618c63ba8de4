"""Real spherical harmonics up to degree 3 in float64 (test infrastructure).

Basis and coefficient order of 3D Gaussian Splatting (the representation the
paper renders, Kerbl et al. 2023): for degree l the functions m = -l .. l are
real SH *with* the Condon-Shortley phase kept, i.e.
    Y_{l,m} = sqrt(2) Im Y_l^{|m|}  (m < 0),  Y_l^0  (m = 0),  sqrt(2) Re Y_l^m  (m > 0),
where Y_l^m are the complex orthonormal harmonics.  The polynomial forms below
are that definition expanded for a unit direction d = (x, y, z); the test suite
checks them against scipy's complex harmonics and by quadrature.

Constants in closed form (pi = math.pi):
  C0 = 1/(2 sqrt(pi)), C1 = sqrt(3)/(2 sqrt(pi)),
  band 2: sqrt(15)/(2 sqrt(pi)), -sqrt(15)/(2 sqrt(pi)), sqrt(5)/(4 sqrt(pi)),
          -sqrt(15)/(2 sqrt(pi)), sqrt(15)/(4 sqrt(pi)),
  band 3: -sqrt(35/2)/(4 sqrt(pi)), sqrt(105)/(2 sqrt(pi)), -sqrt(21/2)/(4 sqrt(pi)),
          sqrt(7)/(4 sqrt(pi)), -sqrt(21/2)/(4 sqrt(pi)), sqrt(105)/(4 sqrt(pi)),
          -sqrt(35/2)/(4 sqrt(pi)).
"""
from __future__ import annotations

import math

import numpy as np

SP = math.sqrt(math.pi)
C0 = 1.0 / (2.0 * SP)
C1 = math.sqrt(3.0) / (2.0 * SP)
C2 = (math.sqrt(15.0) / (2.0 * SP), -math.sqrt(15.0) / (2.0 * SP), math.sqrt(5.0) / (4.0 * SP),
      -math.sqrt(15.0) / (2.0 * SP), math.sqrt(15.0) / (4.0 * SP))
C3 = (-math.sqrt(35.0 / 2.0) / (4.0 * SP), math.sqrt(105.0) / (2.0 * SP), -math.sqrt(21.0 / 2.0) / (4.0 * SP),
      math.sqrt(7.0) / (4.0 * SP), -math.sqrt(21.0 / 2.0) / (4.0 * SP), math.sqrt(105.0) / (4.0 * SP),
      -math.sqrt(35.0 / 2.0) / (4.0 * SP))


def sh_basis(d: np.ndarray, degree: int) -> np.ndarray:
    """Y_k(d) for k < (degree+1)^2; d (..., 3) unit vectors -> (..., K)."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full(x.shape, C0)]
    if degree >= 1:
        out += [-C1 * y, C1 * z, -C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [C2[0] * x * y, C2[1] * y * z, C2[2] * (2.0 * zz - xx - yy), C2[3] * x * z, C2[4] * (xx - yy)]
    if degree >= 3:
        out += [C3[0] * y * (3.0 * xx - yy), C3[1] * x * y * z, C3[2] * y * (4.0 * zz - xx - yy),
                C3[3] * z * (2.0 * zz - 3.0 * xx - 3.0 * yy), C3[4] * x * (4.0 * zz - xx - yy),
                C3[5] * z * (xx - yy), C3[6] * x * (xx - 3.0 * yy)]
    return np.stack(out, axis=-1)


def sh_colour(coeffs: np.ndarray, d: np.ndarray, degree: int) -> np.ndarray:
    """rgb = max(0, 0.5 + sum_k f_k Y_k(d)); coeffs (..., K, 3), d (..., 3) unit.
    (3DGS stores colour with a +0.5 offset on the DC term and clamps at zero;
    there is no upper clamp.)"""
    K = (degree + 1) ** 2
    Y = sh_basis(d, degree)
    c = np.asarray(coeffs, np.float64)[..., :K, :]
    return np.maximum(0.0, 0.5 + np.einsum("...k,...kc->...c", Y, c))
