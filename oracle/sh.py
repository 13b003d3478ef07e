"""Real spherical harmonics of the view direction, FP64 (test infrastructure
only).

The paper feeds the normalised view direction v to the specular network
(Sec. 4.2, Eq. 3) without naming its encoding; the reading adopted is the
real orthonormal spherical-harmonic basis of bands l = 0..3 (16 values), as
in i-NGP's direction encoding.  Index i = l*l + l + m, and

    Y_l^m  = sqrt(2) K_l^m cos(m phi) P_l^m(cos theta)      m > 0
    Y_l^0  =         K_l^0           P_l^0(cos theta)
    Y_l^m  = sqrt(2) K_l^|m| sin(|m| phi) P_l^|m|(cos theta)  m < 0
    K_l^m  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)

with P_l^m the associated Legendre functions including the Condon-Shortley
phase, evaluated here by the standard three-term recurrence in l, and
theta, phi the polar angles of v about +z.

Pins: orthonormality under an exact quadrature (Gauss-Legendre in cos theta
times a uniform rule in phi); the textbook closed forms of bands 0 and 1;
scipy.special's complex harmonics mapped to the real basis.
"""
from __future__ import annotations

import math

import numpy as np


def _legendre(lmax: int, x: np.ndarray):
    """P[l][m](x) for 0 <= m <= l <= lmax, Condon-Shortley phase included."""
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = {}
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = -(2 * m - 1) * s * pmm
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def sh_real(v, degree: int = 4) -> np.ndarray:
    """Real SH of bands 0..degree-1 of directions v [n, 3] (normalised here):
    float64 [n, degree**2]."""
    v = np.asarray(v, np.float64).reshape(-1, 3)
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    lmax = degree - 1
    phi = np.arctan2(v[:, 1], v[:, 0])
    P = _legendre(lmax, np.clip(v[:, 2], -1.0, 1.0))
    out = np.zeros((len(v), degree * degree))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m > 0:
                y = math.sqrt(2.0) * K * np.cos(m * phi) * P[(l, m)]
            elif m < 0:
                y = math.sqrt(2.0) * K * np.sin(am * phi) * P[(l, am)]
            else:
                y = K * P[(l, 0)]
            out[:, l * l + l + m] = y
    return out
