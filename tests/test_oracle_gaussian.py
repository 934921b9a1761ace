"""P2: the oracle's overlap on an atom-centred grid equals closed-form Gaussian overlaps.

Radial functions R(r) = r^l exp(-alpha r^2) (alpha >= 2 / A^2, so truncation at the 4 A
cutoff is below 1e-13), tabulated on 2000 logarithmic knots; product angular rule
(Gauss-Legendre in cos(theta) x uniform phi, 40 x 80), Becke's radial map (200 points) and
full Becke partition weights.  Tolerances come from a convergence study of this very setup
(200-knot tables give ~1e-5, 2000-knot tables ~1e-9 two-centre and ~1e-11 one-centre).
This pins splines, harmonics, the basis assembly and the quadrature together against
mathematics that shares nothing with them.
"""
import math

import numpy as np
import pytest

from oracle import basis as ob
from oracle import integrals as oi
from workloads import generate as g

A = np.array([0.1, -0.2, 0.3])
B = np.array([1.0, 0.5, 1.4])
SHELLS = [[0, 1, 2, 3], [0, 1]]
ALPHAS = [[2.0, 2.5, 3.0, 3.5], [2.2, 2.8]]


@pytest.fixture(scope="module")
def overlap_2000():
    xyz = np.array([A, B])
    desc = g.gaussian_basis(xyz, SHELLS, ALPHAS, 4.0, n_knots=2000)
    X, w, _ = g.make_grid_product(xyz, 4.0, 200, 40, 80)
    return oi.overlap(ob.Basis(desc), X, w)


def _E(al, be):
    p = al + be
    P = (al * A + be * B) / p
    d2 = float(((A - B) ** 2).sum())
    return P, (math.pi / p) ** 1.5 * math.exp(-al * be * d2 / p), p


def test_two_centre_closed_forms(overlap_2000):
    S = overlap_2000
    # basis order: atom 0 -> s(0) p(1..3: y,z,x) d(4..8) f(9..15); atom 1 -> s(16) p(17..19: y,z,x)
    _, E, _ = _E(2.0, 2.2)
    ss = E / (4 * math.pi)
    P, E, _ = _E(2.5, 2.2)
    pxs = math.sqrt(3 / (4 * math.pi)) / (2 * math.sqrt(math.pi)) * (P[0] - A[0]) * E
    pzs = math.sqrt(3 / (4 * math.pi)) / (2 * math.sqrt(math.pi)) * (P[2] - A[2]) * E
    P, E, p = _E(2.5, 2.8)
    pxpx = 3 / (4 * math.pi) * ((P[0] - A[0]) * (P[0] - B[0]) + 1 / (2 * p)) * E
    pxpy = 3 / (4 * math.pi) * ((P[0] - A[0]) * (P[1] - B[1])) * E
    pypz = 3 / (4 * math.pi) * ((P[1] - A[1]) * (P[2] - B[2])) * E
    cases = [(S[0, 16], ss), (S[3, 16], pxs), (S[2, 16], pzs), (S[3, 19], pxpx), (S[3, 17], pxpy),
             (S[1, 18], pypz)]
    for got, ref in cases:
        assert abs(got - ref) <= 2e-9 * abs(ref), (got, ref)


def test_one_centre_closed_forms(overlap_2000):
    S = overlap_2000
    # same-centre: delta_ll' delta_mm' Gamma(l+3/2) / (2 (2 alpha)^(l+3/2))
    blocks = [(0, 1, 0, 2.0), (1, 4, 1, 2.5), (4, 9, 2, 3.0), (9, 16, 3, 3.5)]
    for lo, hi, l, al in blocks:
        ref = math.gamma(l + 1.5) / (2 * (2 * al) ** (l + 1.5))
        assert np.max(np.abs(np.diag(S)[lo:hi] - ref)) <= 1e-10 * ref
    off = S[:16, :16] - np.diag(np.diag(S[:16, :16]))
    # s-d, p-f ... cross terms with different l vanish by orthogonality of Y_lm
    assert np.max(np.abs(off)) <= 1e-12


def test_200_knot_tables_within_spline_error():
    xyz = np.array([A, B])
    desc = g.gaussian_basis(xyz, SHELLS, ALPHAS, 4.0, n_knots=200)
    X, w, _ = g.make_grid_product(xyz, 4.0, 120, 30, 60)
    S = oi.overlap(ob.Basis(desc), X, w)
    _, E, _ = _E(2.0, 2.2)
    assert abs(S[0, 16] - E / (4 * math.pi)) <= 2e-5 * E / (4 * math.pi)
