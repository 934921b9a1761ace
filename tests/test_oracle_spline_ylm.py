"""Pins of the oracle's radial splines and real spherical harmonics against scipy and
textbook identities (independent of the oracle's own formulas)."""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy import special

from oracle import spline as osp
from oracle import ylm as oy


def _samples(n=200, seed=0):
    rng = np.random.default_rng(seed)
    t = np.arange(n, dtype=np.float64)
    return np.sin(0.07 * t) * np.exp(-0.01 * t) + 0.1 * rng.normal(size=n)


def test_spline_matches_scipy_natural():
    y = _samples()
    M = osp.second_derivatives(y)
    cs = CubicSpline(np.arange(len(y), dtype=np.float64), y, bc_type="natural")
    t = np.random.default_rng(1).uniform(0, len(y) - 1, size=5000)
    ours = osp.evaluate_t(t, y, M)
    assert np.max(np.abs(ours - cs(t))) <= 1e-14 * np.max(np.abs(y)) * 10
    # second derivatives at the knots are scipy's
    assert np.max(np.abs(M - cs(np.arange(len(y)), 2))) <= 1e-12 * np.max(np.abs(M))


def test_spline_interpolates_knots_and_natural_ends():
    y = _samples(seed=3)
    M = osp.second_derivatives(y)
    k = np.arange(len(y), dtype=np.float64)
    assert np.max(np.abs(osp.evaluate_t(k, y, M) - y)) <= 1e-15 * np.max(np.abs(y)) * 4
    assert M[0] == 0.0 and M[-1] == 0.0


def test_spline_radial_mapping_and_cutoff():
    rmin, rcut, n = 1e-4, 4.0, 200
    y = _samples(n, seed=5)
    y[-1] = 0.0
    sp = osp.RadialSpline(y, rmin, rcut)
    knots = rmin * (rcut / rmin) ** (np.arange(n) / (n - 1))
    # knots map to integer t, so the spline reproduces the samples there
    assert np.max(np.abs(sp.at_r(knots[:-1]) - y[:-1])) <= 1e-12 * np.max(np.abs(y))
    assert np.all(sp.at_r(np.array([rcut, rcut * 1.5, 100.0])) == 0.0)
    # below rmin the coordinate is clamped to the first knot
    assert sp.at_r(np.array([0.0]))[0] == y[0]
    assert sp.at_r(np.array([1e-6]))[0] == y[0]


def _scipy_real_ylm(l, m, u):
    theta = np.arccos(np.clip(u[:, 2], -1, 1))
    phi = np.arctan2(u[:, 1], u[:, 0])
    Y = special.sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return Y.real
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * Y.real
    return math.sqrt(2.0) * (-1) ** m * Y.imag


def test_ylm_matches_scipy_real_combinations():
    rng = np.random.default_rng(7)
    u = rng.normal(size=(500, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    Y = oy.real_ylm(u)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _scipy_real_ylm(l, m, u)
            assert np.max(np.abs(Y[:, oy.lm_index(l, m)] - ref)) <= 1e-14, (l, m)
    # Y_11 is proportional to +x (no extra Condon-Shortley sign)
    assert oy.real_ylm(np.array([[1.0, 0.0, 0.0]]))[0, oy.lm_index(1, 1)] > 0


def test_ylm_addition_theorem_and_orthonormality():
    rng = np.random.default_rng(9)
    u = rng.normal(size=(300, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    Y = oy.real_ylm(u)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(axis=1)
        assert np.max(np.abs(s - (2 * l + 1) / (4 * math.pi))) <= 1e-14
    # product rule exact for polynomial degree <= 6
    xg, wg = np.polynomial.legendre.leggauss(8)
    nph = 16
    ph = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    z = np.repeat(xg, nph)
    s = np.sqrt(1 - z * z)
    p = np.tile(ph, len(xg))
    uu = np.stack([s * np.cos(p), s * np.sin(p), z], axis=1)
    ww = np.repeat(wg, nph) * 2 * math.pi / nph
    Yq = oy.real_ylm(uu)
    G = Yq.T @ (ww[:, None] * Yq)
    assert np.max(np.abs(G - np.eye(16))) <= 1e-14


@pytest.mark.parametrize("mistake", ["sign_y1", "swap_m"])
def test_ylm_pin_catches_planted_mistakes(mistake, monkeypatch):
    """A planted error in the oracle's harmonics must fail the scipy pin."""
    good = oy.real_ylm

    def bad(u):
        Y = good(u).copy()
        if mistake == "sign_y1":
            Y[..., 1] = -Y[..., 1]
        else:
            Y[..., [4, 8]] = Y[..., [8, 4]]
        return Y

    monkeypatch.setattr(oy, "real_ylm", bad)
    with pytest.raises(AssertionError):
        test_ylm_matches_scipy_real_combinations()
