"""Shared GPU-test inputs: seeded workloads and the oracle's reference values for them.

Every input comes from workloads/ (seeded); every expected value from oracle/.
"""
import functools

import numpy as np

from oracle import basis as ob
from oracle import integrals as oi
from workloads import generate as g


def rel_max(got, ref):
    """Normwise max relative error: max|got - ref| / max|ref|."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    den = float(np.max(np.abs(ref))) if ref.size else 1.0
    return float(np.max(np.abs(got - ref))) / (den if den > 0 else 1.0) if ref.size else 0.0


def _finish(basis, xyz, rp, n_r, n_ang, seed, n_occ, max_batch):
    """Grid, potential and density matrix D = C C^T for a test structure."""
    X, wt, _ = g.make_grid(xyz, rp, n_r, n_ang)
    v = g.gaussian_potential(X, 6, xyz.min(0), xyz.max(0), g.rng_for(7, seed, 2))
    nb = g.n_basis(basis)
    C = g.rng_for(7, seed, 3).normal(size=(nb, n_occ))
    D = C @ C.T
    return dict(basis=basis, xyz=X, w=wt, v=v, D=0.5 * (D + D.T), C=C, max_batch=max_batch, n_basis=nb)


@functools.lru_cache(maxsize=None)
def case(name):
    """Small/medium workloads (oracle runs in seconds) with full oracle references."""
    if name == "config1":
        w = g.config_workload(1)
    elif name == "multitile":
        # a 27-atom config-3-like block (m up to ~380: several 64-wide tiles, ragged tail)
        # on a reduced 16 x 50 grid, batches of <= 256
        xyz = g.geometry_sc_first_n(27, 2.2, 0.1, g.rng_for(3, 100, 0))
        p = dict(g.CONFIGS[3])
        p.update(n_r=16, n_ang=50, n_gauss=16)
        w = g.make_workload(xyz, p, 3, 100, n_occ=40)
    elif name == "two_species":
        xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, -0.4], [0.5, 2.1, 0.7], [3.0, 2.0, 1.0]])
        basis = g.make_basis(xyz, np.array([0, 1, 0, 1], np.int32), [(0, 1, 2, 3), (0, 0, 1)], [4.5, 3.0], 7, 0)
        X, wt, _ = g.make_grid(xyz, 4.5, 14, 50)
        v = g.gaussian_potential(X, 5, xyz.min(0), xyz.max(0), g.rng_for(7, 0, 2))
        nb = g.n_basis(basis)
        C = g.rng_for(7, 0, 3).normal(size=(nb, 6))
        D = C @ C.T
        w = dict(basis=basis, xyz=X, w=wt, v=v, D=0.5 * (D + D.T), C=C, max_batch=64, n_basis=nb)
    elif name == "two_species_8":
        # two species with 8 radial functions each (the shape of a two-element slab basis): a
        # 16 x 200 x 2 knot table, which the basis kernel stages on chip
        xyz = g.geometry_sc_first_n(6, 2.3, 0.1, g.rng_for(7, 8, 0))
        basis = g.make_basis(xyz, np.array([0, 1, 0, 1, 0, 1], np.int32),
                             [(0, 0, 1, 1, 1, 2, 2, 3), (0, 0, 1, 1, 2, 2, 3, 3)], [5.0, 4.0], 7, 8)
        w = _finish(basis, xyz, 5.0, 12, 50, seed=8, n_occ=12, max_batch=128)
    elif name == "dense_cluster":
        # 343 atoms 0.5 A apart with one s function each: the units near the centre see every
        # atom, more than the basis kernel stages on chip
        k = np.arange(7) * 0.5
        xyz = np.array([[x, y, z] for z in k for y in k for x in k])
        basis = g.make_basis(xyz, np.zeros(len(xyz), np.int32), [(0,)], [3.0], 7, 9)
        w = _finish(basis, xyz, 3.0, 2, 6, seed=9, n_occ=30, max_batch=64)
    elif name == "many_species":
        # nine species of 15 shells each: 135 shells, more than the basis kernel stages on chip
        xyz = np.array([[1.6 * i, 1.6 * j, 0.0] for j in range(3) for i in range(3)])
        xyz = xyz + g.rng_for(7, 10, 0).normal(scale=0.1, size=xyz.shape)
        shells = (0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0)
        basis = g.make_basis(xyz, np.arange(9, dtype=np.int32), [shells] * 9, [3.5] * 9, 7, 10)
        w = _finish(basis, xyz, 3.5, 10, 26, seed=10, n_occ=20, max_batch=128)
    else:
        raise KeyError(name)
    B = ob.Basis(w["basis"])
    ref = dict(H=oi.hamiltonian(B, w["xyz"], w["w"], w["v"]),
               S=oi.overlap(B, w["xyz"], w["w"]),
               n=oi.density(B, w["xyz"], w["D"]))
    ref["Ne"] = oi.electron_count(w["w"], ref["n"])
    return w, B, ref


@functools.lru_cache(maxsize=None)
def wide_list_case():
    """150 atoms 0.5 A apart with 32 functions each (4800 functions): the units near the centre
    list every function, more than the density kernel stages the list of on chip (4096).  Only
    the density is referenced (H over 4800 functions costs the oracle minutes)."""
    k = np.arange(6) * 0.5
    xyz = np.array([[x, y, z] for z in k[:5] for y in k[:5] for x in k])
    basis = g.make_basis(xyz, np.zeros(len(xyz), np.int32), [(0, 0, 1, 1, 2, 2, 3, 3)], [4.0], 7, 11)
    w = _finish(basis, xyz, 4.0, 2, 6, seed=11, n_occ=40, max_batch=64)
    B = ob.Basis(w["basis"])
    return w, B, oi.density(B, w["xyz"], w["D"])
