"""Pins for the oracle's SH colour basis (CPU only).

* orthonormality by an exact product quadrature (Gauss-Legendre in cos(theta)
  x uniform in phi is exact for the degree <= 6 products involved);
* every basis function equals (-1)^m times the textbook real harmonic built
  from scipy's complex Y_l^m (a library routine the oracle does not use);
* the polynomial gradient against central differences.
"""
import math

import numpy as np
import scipy.special as sps

from oracle import sh


def _quadrature(nz=8, nphi=16):
    zs, wz = np.polynomial.legendre.leggauss(nz)
    phis = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    Z, PH = np.meshgrid(zs, phis, indexing="ij")
    Wt = (wz[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :])
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(PH), r * np.sin(PH), Z], -1).reshape(-1, 3)
    return d, Wt.reshape(-1)


def test_orthonormal():
    d, w = _quadrature()
    Y = sh.basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_y00_value():
    assert abs(sh.basis(np.array([[0.0, 0.0, 1.0]]), 0)[0, 0] - 1 / (2 * math.sqrt(math.pi))) < 1e-15


def _real_sh_scipy(l, m, d):
    theta = np.arccos(np.clip(d[:, 2], -1, 1))   # polar
    phi = np.arctan2(d[:, 1], d[:, 0])           # azimuth
    if hasattr(sps, "sph_harm_y"):
        Yc = sps.sph_harm_y(l, abs(m), theta, phi)
    else:  # older scipy: sph_harm(m, n, azimuth, polar)
        Yc = sps.sph_harm(abs(m), l, phi, theta)
    if m == 0:
        return Yc.real
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Yc.real
    return math.sqrt(2) * (-1) ** m * Yc.imag


def test_matches_textbook_real_sh():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = sh.basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            ref = (-1) ** m * _real_sh_scipy(l, m, d)
            assert np.abs(Y[:, k] - ref).max() < 1e-12, (l, m)


def test_basis_grad_fd():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(50, 3))
    g = sh.basis_grad(d, 3)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (sh.basis(d + e, 3) - sh.basis(d - e, 3)) / (2 * h)
        assert np.abs(fd - g[:, :, j]).max() < 1e-7


def test_lower_degrees_are_prefixes():
    rng = np.random.default_rng(2)
    d = rng.normal(size=(10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    full = sh.basis(d, 3)
    for deg in range(3):
        assert np.array_equal(sh.basis(d, deg), full[:, :(deg + 1) ** 2])
