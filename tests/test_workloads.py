"""The seeded input generator: determinism, shapes, partition of unity (P11)."""
import math

import numpy as np

from workloads import generate as g


def test_determinism_and_shapes_config1():
    a = g.config_workload(1)
    b = g.config_workload(1)
    for k in ("xyz", "w", "v", "D"):
        assert np.array_equal(a[k], b[k])
    assert a["xyz"].shape == (26400, 3) and a["n_basis"] == 40
    assert np.array_equal(a["D"], a["D"].T)
    assert len(a["basis"]["radial_samples"][0]) == 200


def test_point_counts_and_geometries():
    assert len(g.config_geometry(2)) == 100
    assert len(g.config_geometry(4)) == 375
    p2, p4 = g.CONFIGS[2], g.CONFIGS[4]
    assert 100 * p2["n_r"] * p2["n_ang"] == 1_510_000
    assert 375 * p4["n_r"] * p4["n_ang"] == 9_765_000
    x4 = g.config_geometry(4)
    d = np.sqrt(((x4[:, None] - x4[None]) ** 2).sum(-1)) + np.eye(375) * 99
    assert 2.2 < d.min() < 2.5
    assert np.ptp(x4[:, 2]) > 14.5
    n3 = [len(g.config_geometry(3, s)) for s in range(64)]
    assert min(n3) >= 10 and max(n3) <= 200


def test_becke_native_matches_numpy_reference():
    rng = np.random.default_rng(0)
    atoms = rng.uniform(0, 4, size=(5, 3))
    pts = rng.uniform(-1, 5, size=(300, 3))
    owner = rng.integers(0, 5, size=300).astype(np.int32)
    a = g.becke_owner_weight(atoms, 3.0, pts, owner)
    b = g.becke_owner_weight_numpy(atoms, 3.0, pts, owner)
    assert np.max(np.abs(a - b)) <= 1e-14


def test_p11_partition_of_unity():
    atoms = g.config_geometry(1)
    rng = np.random.default_rng(1)
    probes = rng.uniform(-2, 8, size=(400, 3))
    for r in probes:
        d = np.sqrt(((atoms - r) ** 2).sum(1))
        nb = np.nonzero(d < 4.0)[0]
        if len(nb) == 0:
            continue
        wa = g.becke_owner_weight(atoms, 4.0, np.repeat(r[None], len(nb), 0), nb.astype(np.int32))
        assert abs(wa.sum() - 1.0) <= 1e-14


def test_grid_integrates_normalised_gaussian():
    w = g.config_workload(1, with_density=False)
    c = w["basis"]["atom_xyz"][3]
    a = 1.5
    f = (a / math.pi) ** 1.5 * np.exp(-a * ((w["xyz"] - c) ** 2).sum(1))
    assert abs(np.dot(w["w"], f) - 1.0) <= 2e-3


def test_density_matrix_sparsification():
    x = g.config_workload(2)
    D = x["D"]
    ba = g.basis_atom_index(x["basis"])
    xyz = x["basis"]["atom_xyz"]
    dd = np.sqrt(((xyz[:, None] - xyz[None]) ** 2).sum(-1))
    far = (dd > 10.0)[ba][:, ba]
    assert far.any() and np.all(D[far] == 0.0)
    assert np.array_equal(D, D.T)
