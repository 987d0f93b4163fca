"""Real spherical harmonics up to degree 3 (FP64), the colour basis of a Gaussian.

The paper gives each primitive "colour coefficients" c_i (Sec. 3) without
fixing a basis.  This oracle uses the real SH basis with the Condon-Shortley
phase kept, ordered k = l*l + l + m (m = -l..l):

    Y_k(d) = (-1)^m * Yreal_{l,m}(d)

where Yreal is the textbook real SH (sqrt(2)*Re/Im of the complex Y_l^m with
the CS phase removed).  The normalisation constants below are the closed
forms sqrt((2l+1)/(4 pi) * (l-|m|)!/(l+|m|)!) times the usual polynomial
factors, evaluated here at import time.  Pinned by quadrature orthonormality
and against scipy's complex harmonics in ``tests/test_oracle_sh.py``.
"""
from __future__ import annotations

import math

import numpy as np

_PI = math.pi
_C0 = 1.0 / (2.0 * math.sqrt(_PI))
_C1 = math.sqrt(3.0 / (4.0 * _PI))
_C2a = 0.5 * math.sqrt(15.0 / _PI)      # xy, yz, xz
_C2b = 0.25 * math.sqrt(5.0 / _PI)      # 3z^2 - 1
_C2c = 0.25 * math.sqrt(15.0 / _PI)     # x^2 - y^2
_C3a = 0.25 * math.sqrt(35.0 / (2.0 * _PI))   # y(3x^2-y^2), x(x^2-3y^2)
_C3b = 0.5 * math.sqrt(105.0 / _PI)           # xyz
_C3c = 0.25 * math.sqrt(21.0 / (2.0 * _PI))   # y(5z^2-1), x(5z^2-1)
_C3d = 0.25 * math.sqrt(7.0 / _PI)            # z(5z^2-3)
_C3e = 0.25 * math.sqrt(105.0 / _PI)          # z(x^2-y^2)


def n_coeffs(degree: int) -> int:
    return (degree + 1) ** 2


def basis(d: np.ndarray, degree: int = 3) -> np.ndarray:
    """Y_k(d) for unit directions d [...,3]; returns [..., (degree+1)^2]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full_like(x, _C0)]
    if degree >= 1:
        out += [-_C1 * y, _C1 * z, -_C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [_C2a * x * y, -_C2a * y * z, _C2b * (2.0 * zz - xx - yy),
                -_C2a * x * z, _C2c * (xx - yy)]
    if degree >= 3:
        out += [-_C3a * y * (3.0 * xx - yy), _C3b * x * y * z,
                -_C3c * y * (4.0 * zz - xx - yy), _C3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
                -_C3c * x * (4.0 * zz - xx - yy), _C3e * z * (xx - yy),
                -_C3a * x * (xx - 3.0 * yy)]
    return np.stack(out, axis=-1)


def basis_grad(d: np.ndarray, degree: int = 3) -> np.ndarray:
    """dY_k/d(x,y,z) of the polynomial form (d not renormalised); [..., K, 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    zero = np.zeros_like(x)
    g = [(zero, zero, zero)]
    if degree >= 1:
        g += [(zero, -_C1 + zero, zero), (zero, zero, _C1 + zero), (-_C1 + zero, zero, zero)]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        g += [(_C2a * y, _C2a * x, zero),
              (zero, -_C2a * z, -_C2a * y),
              (-2.0 * _C2b * x, -2.0 * _C2b * y, 4.0 * _C2b * z),
              (-_C2a * z, zero, -_C2a * x),
              (2.0 * _C2c * x, -2.0 * _C2c * y, zero)]
    if degree >= 3:
        g += [(-_C3a * 6.0 * x * y, -_C3a * (3.0 * xx - 3.0 * yy), zero),
              (_C3b * y * z, _C3b * x * z, _C3b * x * y),
              (_C3c * 2.0 * x * y, -_C3c * (4.0 * zz - xx - 3.0 * yy), -_C3c * 8.0 * y * z),
              (-_C3d * 6.0 * x * z, -_C3d * 6.0 * y * z, _C3d * (6.0 * zz - 3.0 * xx - 3.0 * yy)),
              (-_C3c * (4.0 * zz - 3.0 * xx - yy), _C3c * 2.0 * x * y, -_C3c * 8.0 * x * z),
              (_C3e * 2.0 * x * z, -_C3e * 2.0 * y * z, _C3e * (xx - yy)),
              (-_C3a * (3.0 * xx - 3.0 * yy), _C3a * 6.0 * x * y, zero)]
    return np.stack([np.stack(c, axis=-1) for c in g], axis=-2)
