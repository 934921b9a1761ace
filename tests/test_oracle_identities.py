"""Pins of the oracle's quadratures by identities of the method and by brute force.

P3  sum_p w_p n_p = Tr(D S)                 (eq. Density + eq. OverlapNoPeriodic)
P4  Tr(D H) = sum_p w_p v_p n_p             (eq. H_int_aims + eq. Density)
P5  H symmetric
P6  two-atom brute force: (i) triple loop on the same grid, (ii) tensor Gauss-Legendre
    quadrature over the cutoff spheres' box (independent of the partition weights)
P7  batch-size invariance of the batched form (eq. H_decomp)
P8  n = sum_l (sum_i C_il phi_i)^2 for D = C C^T (eq. EVNonPeriodic + eq. DM_from_EV, f = 1)
P13 cell-chunked sums equal octree-batched sums through the nnz(B) lists
P14 zeroing D between centres farther apart than 2 rcut leaves n unchanged (bitwise)
"""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import batching as bt
from oracle import integrals as oi
from workloads import generate as g


@pytest.fixture(scope="module")
def c1():
    w = g.config_workload(1)
    B = ob.Basis(w["basis"])
    H = oi.hamiltonian(B, w["xyz"], w["w"], w["v"])
    S = oi.overlap(B, w["xyz"], w["w"])
    n = oi.density(B, w["xyz"], w["D"])
    return w, B, H, S, n


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def test_p3_electron_count_equals_trace_DS(c1):
    w, B, H, S, n = c1
    Ne = oi.electron_count(w["w"], n)
    assert abs(Ne - float(np.sum(w["D"] * S))) <= 1e-13 * abs(Ne)


def test_p4_trace_DH_equals_weighted_potential_density(c1):
    w, B, H, S, n = c1
    lhs = float(np.sum(w["D"] * H))
    rhs = float(np.dot(w["w"] * w["v"], n))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), float(np.sum(np.abs(w["D"] * H))))


def test_p5_symmetric(c1):
    w, B, H, S, n = c1
    assert np.array_equal(H, H.T) and np.array_equal(S, S.T)


def test_p8_density_from_orbitals(c1):
    w, B, H, S, n = c1
    C = w["C"]
    atoms = np.arange(len(B.atom_xyz))
    Phi = B.phi(w["xyz"], atoms)
    psi = Phi @ C
    ref = (psi ** 2).sum(axis=1)
    assert rel(n, ref) <= 1e-13
    assert np.all(n >= -1e-13 * np.max(n))


def test_density_exact_zero_far_from_atoms(c1):
    w, B, H, S, n = c1
    xyz = w["xyz"]
    d2 = ((xyz[:, None, :] - B.atom_xyz[None, :, :]) ** 2).sum(axis=2)
    far = np.all(d2 >= (B.atom_rcut ** 2)[None, :] * 1.0001, axis=1)
    assert far.sum() > 1000
    assert np.all(n[far] == 0.0)


def test_p13_chunked_equals_batched(c1):
    w, B, H, S, n = c1
    perm, bp = bt.octree_batches(w["xyz"], 200)
    ptr, idx = bt.basis_lists(w["xyz"], perm, bp, B)
    Hb = oi.hamiltonian_batched(B, w["xyz"], w["w"], w["v"], perm, bp, ptr, idx)
    nb = oi.density_batched(B, w["xyz"], w["D"], perm, bp, ptr, idx)
    assert rel(Hb, H) <= 1e-13
    assert rel(nb, n) <= 1e-13


@pytest.mark.parametrize("max_batch", [32, 64, 256])
def test_p7_batch_size_invariance(c1, max_batch):
    w, B, H, S, n = c1
    perm, bp = bt.octree_batches(w["xyz"], max_batch)
    ptr, idx = bt.basis_lists(w["xyz"], perm, bp, B)
    Hb = oi.hamiltonian_batched(B, w["xyz"], w["w"], w["v"], perm, bp, ptr, idx)
    assert rel(Hb, H) <= 1e-13


def test_p6i_two_atom_triple_loop():
    xyz = np.array([[0.0, 0.0, 0.0], [1.7, -0.4, 0.9]])
    desc = g.make_basis(xyz, np.zeros(2, np.int32), [(0, 1)], [3.0], 98, 0)
    B = ob.Basis(desc)
    X, w, _ = g.make_grid(xyz, 3.0, 6, 14)
    v = np.cos(X[:, 0]) + 0.3 * X[:, 1]
    H = oi.hamiltonian(B, X, w, v)
    Phi = B.phi(X, [0, 1])                 # every function at every point, no screening
    nb = Phi.shape[1]
    ref = [[0.0] * nb for _ in range(nb)]
    for p in range(len(X)):
        for i in range(nb):
            for j in range(nb):
                ref[i][j] += w[p] * v[p] * Phi[p, i] * Phi[p, j]
    assert rel(H, np.array(ref)) <= 1e-12


def test_p6ii_two_atom_tensor_quadrature():
    xyz = np.array([[0.0, 0.0, 0.0], [1.3, 0.4, -0.5]])
    rc = 3.0
    B = ob.Basis(g.make_basis(xyz, np.zeros(2, np.int32), [(0, 1, 2)], [rc], 99, 0))

    def vfun(X):
        c = np.array([0.5, 0.2, 0.1])
        return 0.7 * np.exp(-((X - c) ** 2).sum(1) / (2 * 1.1 ** 2)) - 0.3

    X, w, _ = g.make_grid_product(xyz, rc, 150, 30, 60)
    H = oi.hamiltonian(B, X, w, vfun(X))
    lo, hi = xyz.min(0) - rc, xyz.max(0) + rc
    xs, ws = [], []
    for d in range(3):
        x, wg = np.polynomial.legendre.leggauss(60)
        xs.append(lo[d] + (hi[d] - lo[d]) * (x + 1) / 2)
        ws.append(wg * (hi[d] - lo[d]) / 2)
    Xg = np.stack(np.meshgrid(*xs, indexing="ij"), -1).reshape(-1, 3)
    Wg = (ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :]).ravel()
    Phi = B.phi(Xg, [0, 1])
    Ht = Phi.T @ ((Wg * vfun(Xg))[:, None] * Phi)
    # observed 3.0e-6 for this grid (1.5e-5 at 80 x 20 x 40): quadrature error, not rounding
    assert rel(H, Ht) <= 1e-5


def test_p14_sparsified_density_matrix_bitwise():
    xyz = np.array([[2.2 * k, 0.3 * (k % 2), 0.0] for k in range(10)])
    rc = 3.0
    desc = g.make_basis(xyz, np.zeros(10, np.int32), [(0, 1)], [rc], 97, 0)
    B = ob.Basis(desc)
    X, w, _ = g.make_grid(xyz, rc, 8, 26)
    rng = np.random.default_rng(5)
    C = rng.normal(size=(B.n_basis, 6))
    D = C @ C.T
    D = 0.5 * (D + D.T)
    dd = np.sqrt(((xyz[:, None] - xyz[None]) ** 2).sum(-1))
    Dz = D.copy()
    Dz[(dd > 2 * rc)[B.fn_atom][:, B.fn_atom]] = 0.0
    assert np.count_nonzero(D != Dz) > 0
    assert np.array_equal(oi.density(B, X, D), oi.density(B, X, Dz))


def test_density_reads_upper_triangle_only(c1):
    w, B, H, S, n = c1
    D = w["D"].copy()
    D[np.tril_indices(len(D), -1)] = 1e3      # garbage below the diagonal
    assert rel(oi.density(B, w["xyz"], D), n) <= 1e-14


def test_sampled_entry_and_point_helpers(c1):
    w, B, H, S, n = c1
    pairs = [(0, 0), (3, 17), (12, 39), (5, 5)]
    h = oi.hamiltonian_entries(B, w["xyz"], w["w"], w["v"], pairs)
    for k, (i, j) in enumerate(pairs):
        assert abs(h[k] - H[i, j]) <= 1e-13 * np.max(np.abs(H))
    sel = np.arange(0, len(n), 997)
    assert rel(oi.density_at(B, w["xyz"][sel], w["D"]), n[sel]) <= 1e-13


def test_planted_transpose_in_density_fails_p8(c1, monkeypatch):
    """A planted mistake (dropping the j sum: phi_i D_ii phi_i only) must break P8."""
    w, B, H, S, n = c1
    orig = oi.symmetric_from_upper
    monkeypatch.setattr(oi, "symmetric_from_upper", lambda D: np.diag(np.diag(orig(D))))
    bad = oi.density(B, w["xyz"], w["D"])
    C = w["C"]
    psi = B.phi(w["xyz"], np.arange(len(B.atom_xyz))) @ C
    assert rel(bad, (psi ** 2).sum(axis=1)) > 1e-3
