"""Pins of the oracle's density gradient: the spline derivative against scipy, the harmonic
derivatives, grad phi and grad n against central finite differences of the oracle's own phi
and n (which are pinned elsewhere), and a planted mistake that the finite-difference pin
catches."""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import oracle.basis as obm
from oracle import basis as ob
from oracle import integrals as oi
from oracle import spline as osp
from oracle import ylm as oy
from workloads import config_workload
from workloads import generate as g

H = 1e-5


def two_species():
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, -0.4], [0.5, 2.1, 0.7], [3.0, 2.0, 1.0]])
    basis = g.make_basis(xyz, np.array([0, 1, 0, 1], np.int32), [(0, 1, 2, 3), (0, 0, 1)], [4.5, 3.0], 7, 0)
    nb = g.n_basis(basis)
    C = g.rng_for(7, 0, 3).normal(size=(nb, 6))
    return basis, C @ C.T


def sample_points(B, k, seed):
    """Points near the atoms, at least 0.2 A from every nucleus (closer in, the log-grid spline
    varies on the scale of r and central differences with step H lose accuracy)."""
    rng = np.random.default_rng(seed)
    pts = B.atom_xyz[rng.integers(0, len(B.atom_xyz), 4 * k)] + rng.normal(scale=1.3, size=(4 * k, 3))
    dmin = np.sqrt(((pts[:, None, :] - B.atom_xyz[None]) ** 2).sum(-1)).min(axis=1)
    return pts[dmin >= 0.2][:k]


def fd_grad(f, pts):
    out = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = H
        out.append((f(pts + e) - f(pts - e)) / (2 * H))
    return np.stack(out, axis=-1)


def test_spline_derivative_matches_scipy():
    rng = np.random.default_rng(1)
    y = rng.normal(size=40)
    M = osp.second_derivatives(y)
    cs = CubicSpline(np.arange(40.0), y, bc_type="natural").derivative()
    t = rng.uniform(0.0, 39.0, 500)
    assert np.max(np.abs(osp.derivative_t(t, y, M) - cs(t))) <= 1e-12 * np.max(np.abs(cs(t)))


def test_radial_derivative_zero_outside_and_fd_inside():
    rng = np.random.default_rng(2)
    sp = osp.RadialSpline(rng.normal(size=50) * np.linspace(1.0, 0.0, 50), 1e-4, 4.0)
    assert np.all(sp.deriv_at_r(np.array([0.0, 5e-5, 1e-4, 4.0, 4.5])) == 0.0)
    r = rng.uniform(0.05, 3.9, 200)
    fd = (sp.at_r(r + 1e-6) - sp.at_r(r - 1e-6)) / 2e-6
    assert np.max(np.abs(sp.deriv_at_r(r) - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_harmonic_polynomial_derivatives():
    rng = np.random.default_rng(3)
    u = rng.normal(size=(50, 3))  # components independent: not normalised
    G = oy.real_ylm_grad(u)
    fd = np.stack([(oy.real_ylm(u + e) - oy.real_ylm(u - e)) / (2e-6)
                   for e in np.eye(3) * 1e-6], axis=-1)
    assert np.max(np.abs(G - fd)) <= 1e-7 * np.max(np.abs(G))


@pytest.mark.parametrize("case", ["config1", "two_species"])
def test_grad_phi_against_finite_differences(case):
    if case == "config1":
        B = ob.Basis(config_workload(1)["basis"])
    else:
        B = ob.Basis(two_species()[0])
    pts = sample_points(B, 40, 4)
    for a in range(len(B.atom_xyz)):
        G = B.grad_phi_atom(pts, a)
        fd = fd_grad(lambda p: B.phi_atom(p, a), pts)
        assert np.max(np.abs(G - fd)) <= 1e-7 * max(1.0, np.max(np.abs(G)))


@pytest.mark.parametrize("case", ["config1", "two_species"])
def test_density_gradient_against_finite_differences(case):
    if case == "config1":
        w = config_workload(1)
        basis, D = w["basis"], w["D"]
    else:
        basis, D = two_species()
    B = ob.Basis(basis)
    pts = sample_points(B, 30, 5)
    n, grad = oi.density_gradient(B, pts, D, chunks=[np.arange(len(pts))])
    assert np.max(np.abs(n - oi.density_at(B, pts, D))) <= 1e-13 * np.max(np.abs(n))
    fd = fd_grad(lambda p: oi.density_at(B, p, D), pts)
    assert np.max(np.abs(grad - fd)) <= 1e-7 * np.max(np.abs(grad))
    assert np.max(np.abs(oi.density_gradient_at(B, pts, D) - grad)) <= 1e-13 * np.max(np.abs(grad))


def test_chunked_gradient_equals_pointwise():
    w = config_workload(1)
    B = ob.Basis(w["basis"])
    idx = np.arange(0, len(w["xyz"]), 97)
    n, grad = oi.density_gradient(B, w["xyz"][idx], w["D"])
    assert np.max(np.abs(grad - oi.density_gradient_at(B, w["xyz"][idx], w["D"]))) <= 1e-13 * np.max(np.abs(grad))
    far = np.array([[50.0, 50.0, 50.0]])
    assert np.all(oi.density_gradient_at(B, far, w["D"]) == 0.0)


def test_planted_sign_error_in_harmonic_derivative_fails(monkeypatch):
    B = ob.Basis(two_species()[0])
    pts = sample_points(B, 20, 6)
    real = oy.real_ylm_grad

    def wrong(u):
        G = real(u).copy()
        G[..., 2] = -G[..., 2]  # planted: wrong sign of the z derivative
        return G

    monkeypatch.setattr(obm, "real_ylm_grad", wrong)
    G = B.grad_phi_atom(pts, 0)
    fd = fd_grad(lambda p: B.phi_atom(p, 0), pts)
    assert np.max(np.abs(G - fd)) > 1e-3 * np.max(np.abs(G))


def two_atom_case(seed):
    xyz = np.array([[0.0, 0.0, 0.0], [1.7, -0.4, 0.6]])
    basis = g.make_basis(xyz, np.array([0, 0], np.int32), [(0, 1, 2, 3)], [3.5], 11, seed)
    B = ob.Basis(basis)
    X, w, _ = g.make_grid(xyz, 3.5, 8, 26)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=len(X))
    a = rng.normal(size=(len(X), 3))
    return B, X, w, v, a


def test_gga_hamiltonian_reduces_to_local_without_field():
    B, X, w, v, a = two_atom_case(8)
    H0 = oi.hamiltonian(B, X, w, v)
    assert np.max(np.abs(oi.hamiltonian_gga(B, X, w, v, np.zeros_like(a)) - H0)) <= 1e-14 * np.max(np.abs(H0))


def test_gga_hamiltonian_against_pointwise_loops():
    """Independent evaluation: for every point and pair (i, j), the integrand
    w [v phi_i phi_j + a . (grad phi_i phi_j + phi_i grad phi_j)] summed in Python loops."""
    B, X, w, v, a = two_atom_case(9)
    idx = np.arange(0, len(X), 7)
    Xs, ws, vs, as_ = X[idx], w[idx], v[idx], a[idx]
    H = oi.hamiltonian_gga(B, Xs, ws, vs, as_, chunks=[np.arange(len(Xs))])
    atoms = np.arange(len(B.atom_xyz))
    Phi = B.phi(Xs, atoms)
    G = B.grad_phi(Xs, atoms)
    nb = B.n_basis
    ref = np.zeros((nb, nb))
    for p in range(len(Xs)):
        for i in range(nb):
            for j in range(nb):
                gij = G[p, i] * Phi[p, j] + Phi[p, i] * G[p, j]
                ref[i, j] += ws[p] * (vs[p] * Phi[p, i] * Phi[p, j] + float(as_[p] @ gij))
    assert np.max(np.abs(H - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.array_equal(H, H.T)


def test_gga_entries_equal_full_matrix():
    B, X, w, v, a = two_atom_case(10)
    H = oi.hamiltonian_gga(B, X, w, v, a)
    rng = np.random.default_rng(11)
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, B.n_basis, (20, 2))]
    got = oi.hamiltonian_gga_entries(B, X, w, v, a, pairs)
    ref = np.array([H[i, j] for i, j in pairs])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(H))
