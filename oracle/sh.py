"""Real spherical harmonics up to degree 3, built from Legendre polynomials (FP64).

The paper names view-dependent SH colour (Section 2.1) without fixing a basis.
The reading used here is the real orthonormal basis with the Condon-Shortley
phase, indexed b = l*l + (m + l) for m = -l..l:

    Y_lm = sqrt(2) N_l^|m| P_l^|m|(z) cos(m phi)      m > 0
    Y_lm = sqrt(2) N_l^|m| P_l^|m|(z) sin(|m| phi)    m < 0
    Y_l0 = N_l^0 P_l(z)
    N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
    P_l^m(z) = (-1)^m (1 - z^2)^(m/2) d^m/dz^m P_l(z)

On the unit sphere (1 - z^2)^(m/2) cos(m phi) = Re((x + i y)^m) and
(1 - z^2)^(m/2) sin(m phi) = Im((x + i y)^m), so every Y_lm is a polynomial in
(x, y, z).  This module builds those polynomials exactly once (as dicts of
monomial exponents -> coefficient) and evaluates them and their gradients.
Nothing here is a hard-coded table of SH constants.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as _leg
from numpy.polynomial import polynomial as _poly


def _xy_power(m: int):
    """Re and Im of (x + i y)^m as dicts {(i, j): coeff} for x^i y^j."""
    re, im = {}, {}
    for k in range(m + 1):
        c = math.comb(m, k)
        # (i y)^k = i^k y^k
        if k % 2 == 0:
            re[(m - k, k)] = re.get((m - k, k), 0.0) + c * (-1) ** (k // 2)
        else:
            im[(m - k, k)] = im.get((m - k, k), 0.0) + c * (-1) ** ((k - 1) // 2)
    return re, im


def _build(max_degree: int = 3):
    polys = []
    for l in range(max_degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - am) / math.factorial(l + am))
            # d^|m|/dz^|m| P_l as power-series coefficients in z
            dpl = _leg.leg2poly(_leg.legder(np.eye(l + 1)[l], am)) if am <= l else np.zeros(1)
            sign = (-1) ** am
            re, im = _xy_power(am)
            if m == 0:
                xy, scale = {(0, 0): 1.0}, norm
            elif m > 0:
                xy, scale = re, math.sqrt(2.0) * norm
            else:
                xy, scale = im, math.sqrt(2.0) * norm
            poly = {}
            for (i, j), cxy in xy.items():
                for k, cz in enumerate(dpl):
                    if cz == 0.0 or cxy == 0.0:
                        continue
                    key = (i, j, k)
                    poly[key] = poly.get(key, 0.0) + sign * scale * cxy * cz
            polys.append(poly)
    return polys


_POLYS = _build(3)


def num_bases(degree: int) -> int:
    return (degree + 1) ** 2


def eval_sh(degree: int, dirs: np.ndarray, magnitude: bool = False) -> np.ndarray:
    """Y_b(d) for unit directions d [..., 3] -> [..., (degree+1)^2] (FP64).

    magnitude=True: the magnitude companion of each Y_b instead, the sum of the
    absolute values of its polynomial's terms, sum |c| |x|^i |y|^j |z|^k.  Y_b
    is itself a sum of terms that cancel near its nodal lines, so a rounding
    error of a few ulp of those terms is what any evaluation carries there,
    however small Y_b itself is.
    """
    d = np.asarray(dirs, dtype=np.float64)
    if magnitude:
        d = np.abs(d)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = np.zeros(d.shape[:-1] + (num_bases(degree),))
    for b in range(num_bases(degree)):
        acc = np.zeros(d.shape[:-1])
        for (i, j, k), c in _POLYS[b].items():
            acc = acc + (abs(c) if magnitude else c) * x ** i * y ** j * z ** k
        out[..., b] = acc
    return out


def eval_sh_grad(degree: int, dirs: np.ndarray) -> np.ndarray:
    """dY_b/d(x, y, z) of the polynomial extension -> [..., B, 3] (FP64).

    Only the component tangent to the sphere is meaningful; callers project the
    radial part away through the normalisation d = v / |v|.
    """
    d = np.asarray(dirs, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = np.zeros(d.shape[:-1] + (num_bases(degree), 3))

    def pw(t, e):
        return t ** e if e >= 0 else np.zeros_like(t)

    for b in range(num_bases(degree)):
        for (i, j, k), c in _POLYS[b].items():
            if i:
                out[..., b, 0] += c * i * pw(x, i - 1) * pw(y, j) * pw(z, k)
            if j:
                out[..., b, 1] += c * j * pw(x, i) * pw(y, j - 1) * pw(z, k)
            if k:
                out[..., b, 2] += c * k * pw(x, i) * pw(y, j) * pw(z, k - 1)
    return out
