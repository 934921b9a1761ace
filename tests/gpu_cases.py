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
    else:
        raise KeyError(name)
    B = ob.Basis(w["basis"])
    ref = dict(H=oi.hamiltonian(B, w["xyz"], w["w"], w["v"]),
               S=oi.overlap(B, w["xyz"], w["w"]),
               n=oi.density(B, w["xyz"], w["D"]))
    ref["Ne"] = oi.electron_count(w["w"], ref["n"])
    return w, B, ref
