"""Real spherical harmonics up to degree 3 (colour model of Sec. 3.1: a
Gaussian's colour is a function of its SH coefficients and the view
direction).

Convention (a reading; the paper does not fix one): the real basis built from
the complex harmonics with the Condon-Shortley phase,
    m > 0:  sqrt(2) * Re Y_l^m,   m < 0:  sqrt(2) * Im Y_l^|m|,   m = 0: Y_l^0,
ordered by index l*l + l + m.  Written from the definition
    Y_l^m = (-1)^m K_lm P_l^(m)(z) (x + i y)^m,  K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
with P_l^(m) the m-th derivative of the Legendre polynomial P_l, evaluated on
unit directions.  Pinned against scipy.special.sph_harm_y in the tests.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import Legendre

N_COEFFS = 16


def _index(l: int, m: int) -> int:
    return l * l + l + m


def _K(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def basis(d: np.ndarray, degree: int = 3) -> np.ndarray:
    """Real SH basis at unit directions ``d`` (..., 3) -> (..., (degree+1)^2)."""
    d = np.asarray(d, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    w = x + 1j * y
    out = np.zeros(d.shape[:-1] + ((degree + 1) ** 2,))
    for l in range(degree + 1):
        P = Legendre.basis(l)
        for m in range(0, l + 1):
            pz = P.deriv(m)(z) if m > 0 else P(z)
            c = ((-1) ** m) * _K(l, m) * pz * w ** m
            if m == 0:
                out[..., _index(l, 0)] = c.real
            else:
                out[..., _index(l, m)] = math.sqrt(2.0) * c.real
                out[..., _index(l, -m)] = math.sqrt(2.0) * c.imag
    return out


def basis_grad(d: np.ndarray, degree: int = 3) -> np.ndarray:
    """Gradient of the polynomial extension of each basis function with
    respect to (x, y, z): (..., (degree+1)^2, 3).  Only its component tangent
    to the sphere is meaningful; callers project it with the normalisation
    Jacobian."""
    d = np.asarray(d, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    w = x + 1j * y
    out = np.zeros(d.shape[:-1] + ((degree + 1) ** 2, 3))
    for l in range(degree + 1):
        P = Legendre.basis(l)
        for m in range(0, l + 1):
            pz = P.deriv(m)(z) if m > 0 else P(z)
            dpz = P.deriv(m + 1)(z)
            k = ((-1) ** m) * _K(l, m)
            wm = w ** m
            # d/dx w^m = m w^(m-1);  d/dy w^m = i m w^(m-1)
            dw = m * w ** (m - 1) if m > 0 else np.zeros_like(w)
            gx = k * pz * dw
            gy = k * pz * (1j * dw)
            gz = k * dpz * wm
            if m == 0:
                out[..., _index(l, 0), 0] = gx.real
                out[..., _index(l, 0), 1] = gy.real
                out[..., _index(l, 0), 2] = gz.real
            else:
                s = math.sqrt(2.0)
                out[..., _index(l, m), 0] = s * gx.real
                out[..., _index(l, m), 1] = s * gy.real
                out[..., _index(l, m), 2] = s * gz.real
                out[..., _index(l, -m), 0] = s * gx.imag
                out[..., _index(l, -m), 1] = s * gy.imag
                out[..., _index(l, -m), 2] = s * gz.imag
    return out
