"""Real orthonormal spherical harmonics for l <= 3 (oracle).

The angular part of the atom-centred basis functions (eq. EVNonPeriodic's
phi_i = radial x angular; the paper does not state its convention).  Reading:
the standard real combinations of the complex harmonics,
Y_{l,m>0} = sqrt(2) (-1)^m Re Y_l^m, Y_{l,m<0} = sqrt(2) (-1)^m Im Y_l^{|m|},
so that Y_{1,1} is proportional to +x, ordered m = -l..l.  Written out as
polynomials in the unit vector (x, y, z).
"""
from __future__ import annotations

import math

import numpy as np

N_LM = 16  # (l+1)^2 for l <= 3


def real_ylm(u) -> np.ndarray:
    """Y_lm for unit vectors u[..., 3]; returns [..., 16] in order (l, m = -l..l)."""
    u = np.asarray(u, dtype=np.float64)
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    pi = math.pi
    c00 = 0.5 / math.sqrt(pi)
    c1 = math.sqrt(3.0 / (4.0 * pi))
    c2a = 0.5 * math.sqrt(15.0 / pi)
    c2b = 0.25 * math.sqrt(5.0 / pi)
    c2c = 0.25 * math.sqrt(15.0 / pi)
    c3a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
    c3b = 0.5 * math.sqrt(105.0 / pi)
    c3c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
    c3d = 0.25 * math.sqrt(7.0 / pi)
    c3e = 0.25 * math.sqrt(105.0 / pi)
    out = [
        np.full_like(x, c00),
        c1 * y, c1 * z, c1 * x,
        c2a * x * y, c2a * y * z, c2b * (3.0 * z * z - 1.0), c2a * x * z, c2c * (x * x - y * y),
        c3a * y * (3.0 * x * x - y * y), c3b * x * y * z, c3c * y * (5.0 * z * z - 1.0),
        c3d * (5.0 * z ** 3 - 3.0 * z), c3c * x * (5.0 * z * z - 1.0), c3e * z * (x * x - y * y),
        c3a * x * (x * x - 3.0 * y * y),
    ]
    return np.stack(out, axis=-1)


def real_ylm_grad(u) -> np.ndarray:
    """Partial derivatives of the polynomials of real_ylm with respect to the three
    components of u, taken as independent variables: [..., 16, 3]."""
    u = np.asarray(u, dtype=np.float64)
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    pi = math.pi
    c1 = math.sqrt(3.0 / (4.0 * pi))
    c2a = 0.5 * math.sqrt(15.0 / pi)
    c2b = 0.25 * math.sqrt(5.0 / pi)
    c2c = 0.25 * math.sqrt(15.0 / pi)
    c3a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
    c3b = 0.5 * math.sqrt(105.0 / pi)
    c3c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
    c3d = 0.25 * math.sqrt(7.0 / pi)
    c3e = 0.25 * math.sqrt(105.0 / pi)
    o = np.zeros_like(x)
    rows = [
        (o, o, o),
        (o, c1 + o, o), (o, o, c1 + o), (c1 + o, o, o),
        (c2a * y, c2a * x, o), (o, c2a * z, c2a * y), (o, o, 6.0 * c2b * z), (c2a * z, o, c2a * x),
        (2.0 * c2c * x, -2.0 * c2c * y, o),
        (6.0 * c3a * x * y, c3a * (3.0 * x * x - 3.0 * y * y), o),
        (c3b * y * z, c3b * x * z, c3b * x * y),
        (o, c3c * (5.0 * z * z - 1.0), 10.0 * c3c * y * z),
        (o, o, c3d * (15.0 * z * z - 3.0)),
        (c3c * (5.0 * z * z - 1.0), o, 10.0 * c3c * x * z),
        (2.0 * c3e * x * z, -2.0 * c3e * y * z, c3e * (x * x - y * y)),
        (c3a * (3.0 * x * x - 3.0 * y * y), -6.0 * c3a * x * y, o),
    ]
    return np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)


def lm_index(l: int, m: int) -> int:
    return l * l + (m + l)
