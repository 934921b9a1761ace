"""Pins of the oracle's kinetic term: the spline's second derivative against scipy, the
Laplacian of the basis functions against central finite differences of phi and against the
closed forms for Gaussian s and p functions, the kinetic matrix against its integrated-by-parts
form (1/2) sum_p w grad phi_i . grad phi_j, and the decomposition of the Kohn-Sham matrix into
the kinetic, local and vector-field parts (each pinned elsewhere)."""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import basis as ob
from oracle import integrals as oi
from oracle import spline as osp
from oracle import ylm as oy
from workloads import config_workload
from workloads import generate as g

STEP = 1e-4


def two_species():
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, -0.4], [0.5, 2.1, 0.7], [3.0, 2.0, 1.0]])
    return g.make_basis(xyz, np.array([0, 1, 0, 1], np.int32), [(0, 1, 2, 3), (0, 0, 1)], [4.5, 3.0], 7, 0)


def sample_points(B, k, seed):
    """Points near the atoms, at least 0.2 A from every nucleus."""
    rng = np.random.default_rng(seed)
    pts = B.atom_xyz[rng.integers(0, len(B.atom_xyz), 4 * k)] + rng.normal(scale=1.3, size=(4 * k, 3))
    dmin = np.sqrt(((pts[:, None, :] - B.atom_xyz[None]) ** 2).sum(-1)).min(axis=1)
    return pts[dmin >= 0.2][:k]


def test_spline_second_derivative_matches_scipy():
    rng = np.random.default_rng(1)
    y = rng.normal(size=40)
    M = osp.second_derivatives(y)
    cs = CubicSpline(np.arange(40.0), y, bc_type="natural").derivative(2)
    t = rng.uniform(0.0, 39.0, 500)
    assert np.max(np.abs(osp.second_t(t, y, M) - cs(t))) <= 1e-12 * np.max(np.abs(cs(t)))


@pytest.mark.parametrize("case", ["config1", "two_species"])
def test_laplacian_against_finite_differences(case):
    B = ob.Basis(config_workload(1)["basis"] if case == "config1" else two_species())
    pts = sample_points(B, 40, 4)
    for a in range(len(B.atom_xyz)):
        lap = B.lap_phi_atom(pts, a)
        fd = -6.0 * B.phi_atom(pts, a)
        for e in np.eye(3) * STEP:
            fd = fd + B.phi_atom(pts + e, a) + B.phi_atom(pts - e, a)
        fd = fd / (STEP * STEP)
        assert np.max(np.abs(lap - fd)) <= 1e-5 * max(1.0, np.max(np.abs(lap)))


def test_laplacian_gaussian_closed_forms():
    """R = exp(-alpha r^2) (l = 0) and R = r exp(-alpha r^2) (l = 1): lap phi =
    Y (4 alpha^2 r^2 - 6 alpha) exp(-alpha r^2) and Y r (4 alpha^2 r^2 - 10 alpha) exp(-alpha r^2)."""
    alpha, rmin, rcut, n = 1.3, 1e-4, 8.0, 1500
    r_k = rmin * np.exp(np.arange(n) * (math.log(rcut / rmin) / (n - 1)))
    desc = dict(atom_xyz=np.zeros((1, 3)), atom_species=np.zeros(1, np.int32),
                species_shell_ptr=np.array([0, 2], np.int32), shell_l=np.array([0, 1], np.int32),
                shell_radial=np.array([0, 1], np.int32), radial_rmin=np.array([rmin, rmin]),
                radial_rcut=np.array([rcut, rcut]),
                radial_samples=np.stack([np.exp(-alpha * r_k ** 2), r_k * np.exp(-alpha * r_k ** 2)]),
                n_knots=n)
    B = ob.Basis(desc)
    rng = np.random.default_rng(5)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = rng.uniform(0.1, 3.0, 300)
    pts = d * r[:, None]
    Y = oy.real_ylm(d)
    gauss = np.exp(-alpha * r * r)
    ref = np.stack([Y[:, 0] * (4 * alpha ** 2 * r * r - 6 * alpha) * gauss]
                   + [Y[:, k] * r * (4 * alpha ** 2 * r * r - 10 * alpha) * gauss for k in (1, 2, 3)], axis=1)
    lap = B.lap_phi_atom(pts, 0)
    assert np.max(np.abs(lap - ref)) <= 1e-4 * np.max(np.abs(ref))


def two_atom_case(seed, n_r=40, n_ang=110):
    xyz = np.array([[0.0, 0.0, 0.0], [1.7, -0.4, 0.6]])
    basis = g.make_basis(xyz, np.array([0, 0], np.int32), [(0, 1, 2, 3)], [3.5], 11, seed)
    B = ob.Basis(basis)
    X, w, _ = g.make_grid(xyz, 3.5, n_r, n_ang)
    rng = np.random.default_rng(seed)
    return B, X, w, rng.normal(size=len(X)), rng.normal(size=(len(X), 3))


def test_kinetic_matches_integrated_by_parts_form():
    """The radial functions vanish with their derivatives at the cutoff, so
    -1/2 int phi_i lap phi_j = 1/2 int grad phi_i . grad phi_j up to the grid's quadrature error
    (9.7e-4 normwise on this 80 x 302 grid, 8e-3 on 40 x 110: the angular grid dominates)."""
    B, X, w, v, a = two_atom_case(21, 80, 302)
    T = oi.kinetic(B, X, w)
    atoms = np.arange(len(B.atom_xyz))
    G = B.grad_phi(X, atoms)
    ref = 0.5 * np.einsum("pik,pjk->ij", w[:, None, None] * G, G)
    assert np.max(np.abs(T - ref)) <= 2e-3 * np.max(np.abs(ref))
    assert np.all(np.linalg.eigvalsh(ref) > -1e-9 * np.max(np.abs(ref)))


def test_ks_hamiltonian_decomposes():
    B, X, w, v, a = two_atom_case(22)
    idx = np.arange(0, len(X), 5)
    X, w, v, a = X[idx], w[idx], v[idx], a[idx]
    H = oi.hamiltonian_ks(B, X, w, v, a)
    ref = oi.hamiltonian_gga(B, X, w, v, a) + oi.kinetic(B, X, w)
    assert np.max(np.abs(H - ref)) <= 1e-12 * np.max(np.abs(ref))
    ref0 = oi.hamiltonian(B, X, w, v) + oi.kinetic(B, X, w)
    assert np.max(np.abs(oi.hamiltonian_ks(B, X, w, v) - ref0)) <= 1e-12 * np.max(np.abs(ref0))


def test_ks_entries_equal_full_matrix():
    B, X, w, v, a = two_atom_case(23)
    idx = np.arange(0, len(X), 5)
    X, w, v, a = X[idx], w[idx], v[idx], a[idx]
    rng = np.random.default_rng(24)
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, B.n_basis, (20, 2))]
    for field in (a, None):
        H = oi.hamiltonian_ks(B, X, w, v, field)
        got = oi.hamiltonian_ks_entries(B, X, w, v, field, pairs)
        assert np.max(np.abs(got - np.array([H[i, j] for i, j in pairs]))) <= 1e-12 * np.max(np.abs(H))


def test_planted_dropped_angular_term_fails(monkeypatch):
    """A Laplacian without the -l(l+1) R / r^2 term must fail the finite-difference pin."""
    B = ob.Basis(two_species())
    pts = sample_points(B, 30, 7)
    real = osp.radial_laplacian

    def wrong(r, y, M, rmin, rcut, l):
        return real(r, y, M, rmin, rcut, 0)  # planted: angular term dropped

    monkeypatch.setattr(osp, "radial_laplacian", wrong)
    lap = B.lap_phi_atom(pts, 0)
    fd = -6.0 * B.phi_atom(pts, 0)
    for e in np.eye(3) * STEP:
        fd = fd + B.phi_atom(pts + e, 0) + B.phi_atom(pts - e, 0)
    fd = fd / (STEP * STEP)
    assert np.max(np.abs(lap - fd)) > 1e-3 * np.max(np.abs(fd))
