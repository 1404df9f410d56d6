"""Pins of the oracle's real spherical harmonics (oracle/sh.py)."""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import sh


def _dirs(n, seed=0):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_y00():
    Y = sh.eval_sh(0, _dirs(4))
    assert np.allclose(Y[:, 0], 1.0 / (2.0 * math.sqrt(math.pi)), rtol=0, atol=1e-16)


def test_sum_rule_unsold():
    # sum_m Y_lm(d)^2 = (2l+1)/(4 pi) for every direction, under any sign convention
    Y = sh.eval_sh(3, _dirs(200, 1))
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        assert np.allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-13, atol=0)


def test_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi: exact for the degree-6 products
    zs, wz = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phis = 2 * math.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(zs, phis, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(PHI), r * np.sin(PHI), Z], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y = sh.eval_sh(3, d)
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-13)


def test_matches_scipy_complex_harmonics():
    # real basis from scipy's complex Y_l^m (Condon-Shortley phase included):
    # m > 0: sqrt(2) Re Y_l^m, m < 0: sqrt(2) Im Y_l^|m|, m = 0: Y_l^0
    d = _dirs(50, 2)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = sh.eval_sh(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            c = sps.sph_harm_y(l, abs(m), theta, phi)
            ref = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
            assert np.allclose(Y[:, l * l + m + l], ref, atol=1e-13), (l, m)


def test_gradient_tangential_fd():
    d = _dirs(20, 3)
    G = sh.eval_sh_grad(3, d)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        fd = (sh.eval_sh(3, d + h * e) - sh.eval_sh(3, d - h * e)) / (2 * h)
        assert np.allclose(G[:, :, k], fd, atol=1e-8)


def test_magnitude_companion_bounds_the_value_and_float32_rounding():
    # the companion sums |term| of each Y_b's polynomial: it is >= |Y_b|, equal
    # to it for l <= 1 (one monomial each), and a
    # float32 evaluation of the same polynomial stays within a few ulp of it
    # even on nodal lines, where |Y_b| itself gives no scale
    d = _dirs(4000, 7)
    Y = sh.eval_sh(3, d)
    M = sh.eval_sh(3, d, magnitude=True)
    assert np.all(M >= np.abs(Y) * (1 - 1e-15))
    assert np.allclose(M[:, :4], np.abs(Y[:, :4]), rtol=1e-15, atol=0)
    # float32 evaluation: every product and sum rounded to float32
    d32 = d.astype(np.float32)
    x, y, z = d32[:, 0], d32[:, 1], d32[:, 2]
    err_rel_M, err_rel_Y = 0.0, 0.0
    for b in range(16):
        acc = np.zeros(d.shape[0], np.float32)
        for (i, j, k), c in sh._POLYS[b].items():
            acc = (acc + np.float32(c) * x ** i * y ** j * z ** k).astype(np.float32)
        e = np.abs(acc.astype(np.float64) - Y[:, b])
        err_rel_M = max(err_rel_M, float((e / M[:, b]).max()))
        err_rel_Y = max(err_rel_Y, float((e / np.abs(Y[:, b])).max()))
    assert err_rel_M < 2e-6
    # (near nodal lines the error relative to |Y_b| is far larger)
    assert err_rel_Y > 1e-4
