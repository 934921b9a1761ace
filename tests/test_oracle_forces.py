"""Pins of the oracle's local Pulay forces (h_KS = t + v).

* The local-potential and q parts: central finite differences of the oracle's own Hamiltonian and
  overlap (pinned elsewhere) under a displacement of one atom's basis functions.
* The kinetic part, -2 sum_ij sum_p w [grad_A phi_i] n_ij (-lap phi_j / 2): central finite
  differences of sum_ij n_ij sum_p w phi_i (-lap phi_j / 2) with only the left factor's atom
  displaced (the pinned phi and lap phi), an exact identity on the grid.  The paper's form stands
  for twice this derivative because t is Hermitian; on a finite grid that holds up to the
  quadrature error of integrating by parts, which shrinks as the grid is refined.
* The sum over atoms against the (pinned) density gradient, the per-atom sampled form against
  the full one, and planted mistakes that the finite-difference pins catch."""
import copy

import numpy as np
import pytest

from oracle import basis as ob
from oracle import integrals as oi
from workloads import config_workload
from workloads import generate as g

STEP = 1e-5


def case(seed, species=(0, 0), xyz=((0.0, 0.0, 0.0), (1.7, -0.4, 0.6))):
    xyz = np.array(xyz, dtype=np.float64)
    basis = g.make_basis(xyz, np.array(species, np.int32), [(0, 1, 2, 3), (0, 0, 1)][:max(species) + 1],
                         [3.5, 2.8][:max(species) + 1], 11, seed)
    X, w, _ = g.make_grid(xyz, 3.5, 8, 26)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=len(X))
    nb = g.n_basis(basis)
    C = rng.normal(size=(nb, 5))
    D = C @ C.T
    C2 = rng.normal(size=(nb, 5))
    Q = C2 @ np.diag(rng.normal(size=5)) @ C2.T
    return basis, X, w, v, D, Q


def energy(desc, X, w, v, D, Q):
    """E = sum_ij D_ij h_ij - sum_ij Q_ij s_ij with the grid, weights and v held fixed."""
    B = ob.Basis(desc)
    return float(np.sum(D * oi.hamiltonian(B, X, w, v)) - np.sum(Q * oi.overlap(B, X, w)))


def fd_forces(basis, X, w, v, D, Q):
    n_at = len(np.asarray(basis["atom_xyz"]).reshape(-1, 3))
    F = np.zeros((n_at, 3))
    for A in range(n_at):
        for k in range(3):
            moved = []
            for sgn in (1.0, -1.0):
                d = copy.deepcopy(basis)
                x = np.array(d["atom_xyz"], dtype=np.float64).reshape(-1, 3)
                x[A, k] += sgn * STEP
                d["atom_xyz"] = x
                moved.append(energy(d, X, w, v, D, Q))
            F[A, k] = -(moved[0] - moved[1]) / (2 * STEP)
    return F


@pytest.mark.parametrize("kind", ["one_species", "two_species"])
def test_forces_against_finite_differences(kind):
    if kind == "one_species":
        basis, X, w, v, D, Q = case(12)
    else:
        basis, X, w, v, D, Q = case(13, (0, 1, 0), ((0.0, 0.0, 0.0), (1.9, 0.3, -0.4), (0.5, 2.1, 0.7)))
    F = oi.pulay_forces(ob.Basis(basis), X, w, v, D, Q, kinetic=False)
    fd = fd_forces(basis, X, w, v, D, Q)
    assert np.max(np.abs(F - fd)) <= 1e-7 * np.max(np.abs(F))


def kinetic_left(desc_left, desc, X, w, D):
    """sum_ij n_ij sum_p w_p phi_i(r_p) (-lap phi_j(r_p) / 2), phi_i from desc_left."""
    BL, B = ob.Basis(desc_left), ob.Basis(desc)
    every = np.arange(len(B.atom_xyz))
    PL = BL.phi(X, every)
    LP = B.lap_phi(X, every)
    return float(np.sum(oi.symmetric_from_upper(D) * (PL.T @ (-0.5 * w[:, None] * LP))))


def fd_kinetic(basis, X, w, D):
    """-2 d/dR_A of kinetic_left with only the left factor's atom A displaced."""
    n_at = len(np.asarray(basis["atom_xyz"]).reshape(-1, 3))
    F = np.zeros((n_at, 3))
    for A in range(n_at):
        for k in range(3):
            moved = []
            for sgn in (1.0, -1.0):
                d = copy.deepcopy(basis)
                x = np.array(d["atom_xyz"], dtype=np.float64).reshape(-1, 3)
                x[A, k] += sgn * STEP
                d["atom_xyz"] = x
                moved.append(kinetic_left(d, basis, X, w, D))
            F[A, k] = -2.0 * (moved[0] - moved[1]) / (2 * STEP)
    return F


@pytest.mark.parametrize("kind", ["one_species", "two_species"])
def test_kinetic_part_against_finite_differences(kind):
    if kind == "one_species":
        basis, X, w, v, D, Q = case(18)
    else:
        basis, X, w, v, D, Q = case(19, (0, 1, 0), ((0.0, 0.0, 0.0), (1.9, 0.3, -0.4), (0.5, 2.1, 0.7)))
    B = ob.Basis(basis)
    F_kin = oi.pulay_forces(B, X, w, v, D, Q) - oi.pulay_forces(B, X, w, v, D, Q, kinetic=False)
    fd = fd_kinetic(basis, X, w, D)
    assert np.max(np.abs(fd)) > 1e-2 * np.max(np.abs(oi.pulay_forces(B, X, w, v, D, Q)))  # not negligible
    assert np.max(np.abs(F_kin - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_planted_kinetic_sign_fails(monkeypatch):
    """A kinetic operator of the wrong sign (+lap / 2) fails the kinetic pin."""
    basis, X, w, v, D, Q = case(20)
    B = ob.Basis(basis)
    real = B.lap_phi
    monkeypatch.setattr(B, "lap_phi", lambda pts, atoms: -real(pts, atoms))  # planted: t = +lap / 2
    F_kin = oi.pulay_forces(B, X, w, v, D, Q) - oi.pulay_forces(B, X, w, v, D, Q, kinetic=False)
    fd = fd_kinetic(basis, X, w, D)
    assert np.max(np.abs(F_kin - fd)) > 1e-1 * np.max(np.abs(fd))


def test_force_sum_equals_weighted_density_gradients():
    """Local-potential and q parts: sum_A F_A = sum_p w_p [v_p grad n_D(r_p) - grad n_Q(r_p)], n_X
    the density of matrix X."""
    basis, X, w, v, D, Q = case(14)
    B = ob.Basis(basis)
    F = oi.pulay_forces(B, X, w, v, D, Q, kinetic=False)
    _, gD = oi.density_gradient(B, X, D)
    _, gQ = oi.density_gradient(B, X, Q)
    ref = ((w * v)[:, None] * gD - w[:, None] * gQ).sum(axis=0)
    assert np.max(np.abs(F.sum(axis=0) - ref)) <= 1e-12 * np.max(np.abs(F))


def test_sampled_atoms_equal_full_forces():
    w_ = config_workload(1)
    B = ob.Basis(w_["basis"])
    rng = np.random.default_rng(15)
    Q = w_["D"] * 0.3 + np.diag(rng.normal(size=B.n_basis))
    F = oi.pulay_forces(B, w_["xyz"], w_["w"], w_["v"], w_["D"], Q)
    atoms = [0, 3, 7]
    got = oi.pulay_forces_at(B, w_["xyz"], w_["w"], w_["v"], w_["D"], Q, atoms)
    assert np.max(np.abs(got - F[atoms])) <= 1e-12 * np.max(np.abs(F))


def test_only_upper_triangles_are_read():
    basis, X, w, v, D, Q = case(16)
    B = ob.Basis(basis)
    F = oi.pulay_forces(B, X, w, v, D, Q)
    junk = np.tril(np.full_like(D, 1e3), -1)
    assert np.array_equal(oi.pulay_forces(B, X, w, v, np.triu(D) + junk, np.triu(Q) - junk), F)


def test_planted_swapped_gradient_components_fail(monkeypatch):
    basis, X, w, v, D, Q = case(17)
    B = ob.Basis(basis)
    real = B.grad_phi

    def wrong(pts, atoms):
        return real(pts, atoms)[:, :, [1, 0, 2]]  # planted: x and y derivatives swapped

    monkeypatch.setattr(B, "grad_phi", wrong)
    F = oi.pulay_forces(B, X, w, v, D, Q, kinetic=False)
    fd = fd_forces(basis, X, w, v, D, Q)
    assert np.max(np.abs(F - fd)) > 1e-3 * np.max(np.abs(fd))
