"""Radial functions as natural cubic splines on a logarithmic grid (oracle).

The paper's basis functions are numeric atom-centred orbitals whose radial
parts vanish beyond a confining radius (Section "Computational Choices in
FHI-aims"); it does not state how they are tabulated.  Reading used here:

* knots r_k = rmin (rcut/rmin)^(k/(N-1)), k = 0..N-1; spline variable
  t = ln(r/rmin)/Delta with Delta = ln(rcut/rmin)/(N-1), so knot k sits at t = k;
* natural boundary conditions: M_0 = M_{N-1} = 0 and, for 0 < k < N-1,
  M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1}),
  where M_k is the second derivative in t;
* evaluation: R = 0 outside the cutoff; otherwise t is clamped to [0, N-1],
  k = min(floor(t), N-2), u = t - k and
  R = (1-u) y_k + u y_{k+1} + (((1-u)^3 - (1-u)) M_k + (u^3 - u) M_{k+1}) / 6.

Radial derivative (for density gradients): dR/dr = (dR/dt) / (r Delta) for
rmin < r < rcut, with dR/dt the derivative of the evaluation formula in u; the
spline is constant in the clamped region r <= rmin, so dR/dr = 0 there, and
dR/dr = 0 at and beyond the cutoff.

Radial part of the Laplacian (for the kinetic term): for phi = R(r) Y_lm(unit r),
lap phi = (R'' + 2 R'/r - l(l+1) R/r^2) Y_lm; with R' = S'/(Delta r) and
R'' = (S'' - Delta S')/(Delta r)^2 in the spline variable this is
(S''/Delta^2 + S'/Delta - l(l+1) S) / r^2, where S'' = (1-u) M_k + u M_{k+1} is the
spline's own (piecewise linear) second derivative.  Reading: zero for r <= rmin
and r >= rcut, like the derivative.

Plain Python loops for the tridiagonal solve (Thomas algorithm).
"""
from __future__ import annotations

import math

import numpy as np


def second_derivatives(y) -> np.ndarray:
    """M_k of the natural cubic spline through y_k at unit-spaced t = k."""
    y = [float(v) for v in y]
    n = len(y)
    if n < 4:
        raise ValueError("need at least 4 knots")
    m = n - 2  # unknowns M_1..M_{n-2}
    diag = [4.0] * m
    rhs = [6.0 * (y[k - 1] - 2.0 * y[k] + y[k + 1]) for k in range(1, n - 1)]
    # forward elimination (sub- and super-diagonals are 1)
    for i in range(1, m):
        f = 1.0 / diag[i - 1]
        diag[i] -= f
        rhs[i] -= f * rhs[i - 1]
    M = [0.0] * m
    M[m - 1] = rhs[m - 1] / diag[m - 1]
    for i in range(m - 2, -1, -1):
        M[i] = (rhs[i] - M[i + 1]) / diag[i]
    return np.array([0.0] + M + [0.0])


def spline_t(r, rmin: float, rcut: float, n_knots: int) -> np.ndarray:
    """Spline coordinate t = ln(r/rmin)/Delta, clamped to [0, N-1] (r <= rmin gives 0)."""
    r = np.asarray(r, dtype=np.float64)
    delta = math.log(rcut / rmin) / (n_knots - 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(r > rmin, np.log(np.where(r > rmin, r, rmin) / rmin) / delta, 0.0)
    return np.clip(t, 0.0, float(n_knots - 1))


def evaluate_t(t, y, M) -> np.ndarray:
    """Cubic spline value at (already clamped) coordinate t."""
    t = np.asarray(t, dtype=np.float64)
    n = len(y)
    k = np.minimum(np.floor(t).astype(np.int64), n - 2)
    u = t - k
    a = 1.0 - u
    return a * y[k] + u * y[k + 1] + ((a ** 3 - a) * M[k] + (u ** 3 - u) * M[k + 1]) / 6.0


def derivative_t(t, y, M) -> np.ndarray:
    """dR/dt of the cubic spline at (already clamped) coordinate t."""
    t = np.asarray(t, dtype=np.float64)
    n = len(y)
    k = np.minimum(np.floor(t).astype(np.int64), n - 2)
    u = t - k
    a = 1.0 - u
    # d/du of a y_k + u y_{k+1} + ((a^3 - a) M_k + (u^3 - u) M_{k+1}) / 6, with da/du = -1
    return (y[k + 1] - y[k]) + ((1.0 - 3.0 * a * a) * M[k] + (3.0 * u * u - 1.0) * M[k + 1]) / 6.0


def second_t(t, y, M) -> np.ndarray:
    """d^2R/dt^2 of the cubic spline at (already clamped) coordinate t."""
    t = np.asarray(t, dtype=np.float64)
    n = len(y)
    k = np.minimum(np.floor(t).astype(np.int64), n - 2)
    u = t - k
    return (1.0 - u) * M[k] + u * M[k + 1]


def radial_laplacian(r, y, M, rmin: float, rcut: float, l: int) -> np.ndarray:
    """R'' + 2 R'/r - l(l+1) R/r^2: zero for r <= rmin and for r >= rcut."""
    r = np.asarray(r, dtype=np.float64)
    n = len(y)
    delta = math.log(rcut / rmin) / (n - 1)
    inside = (r > rmin) & (r < rcut)
    safe = np.where(inside, r, 1.0)
    t = spline_t(safe, rmin, rcut, n)
    S = evaluate_t(t, y, M)
    dS = derivative_t(t, y, M)
    d2S = second_t(t, y, M)
    val = (d2S / (delta * delta) + dS / delta - l * (l + 1) * S) / (safe * safe)
    return np.where(inside, val, 0.0)


def radial_derivative(r, y, M, rmin: float, rcut: float) -> np.ndarray:
    """dR/dr: zero for r <= rmin (clamped, constant) and for r >= rcut."""
    r = np.asarray(r, dtype=np.float64)
    n = len(y)
    delta = math.log(rcut / rmin) / (n - 1)
    inside = (r > rmin) & (r < rcut)
    safe = np.where(inside, r, 1.0)
    dt = derivative_t(spline_t(safe, rmin, rcut, n), y, M)
    return np.where(inside, dt / (safe * delta), 0.0)


class RadialSpline:
    """One tabulated radial function R(r) on the logarithmic grid."""

    def __init__(self, samples, rmin: float, rcut: float):
        self.y = np.asarray(samples, dtype=np.float64)
        self.M = second_derivatives(self.y)
        self.rmin = float(rmin)
        self.rcut = float(rcut)
        self.n = len(self.y)

    def at_r(self, r) -> np.ndarray:
        """R(r) with R = 0 for r >= rcut (used by the spline pins)."""
        r = np.asarray(r, dtype=np.float64)
        val = evaluate_t(spline_t(r, self.rmin, self.rcut, self.n), self.y, self.M)
        return np.where(r >= self.rcut, 0.0, val)

    def deriv_at_r(self, r) -> np.ndarray:
        """dR/dr (zero for r <= rmin and r >= rcut)."""
        return radial_derivative(r, self.y, self.M, self.rmin, self.rcut)

    def laplacian_at_r(self, r, l: int) -> np.ndarray:
        """R'' + 2 R'/r - l(l+1) R/r^2 (zero for r <= rmin and r >= rcut)."""
        return radial_laplacian(r, self.y, self.M, self.rmin, self.rcut, l)
