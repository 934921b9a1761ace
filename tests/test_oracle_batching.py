"""P12: the oracle's octree batches and nnz(B) lists against independent brute force.

The batches are re-derived from per-point octant paths (repeated halving of the root box):
a point's batch is the shortest path prefix whose node holds <= max_batch points, and
depth-first pre-order equals lexicographic order of the paths.  The lists are checked for
completeness through the basis functions themselves (every non-zero phi_i(r_p) is listed
for p's batch) and for minimality through distances.
"""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import batching as bt
from workloads import generate as g


def brute_force_batches(xyz, max_batch, max_depth=bt.MAX_DEPTH):
    n = len(xyz)
    lo = np.tile(xyz.min(axis=0), (n, 1))
    hi = np.tile(xyz.max(axis=0), (n, 1))
    paths = np.zeros((n, max_depth), dtype=np.int64)
    counts = []
    for d in range(max_depth):
        mid = 0.5 * (lo + hi)
        bits = xyz >= mid
        paths[:, d] = bits[:, 0] + 2 * bits[:, 1] + 4 * bits[:, 2]
        lo = np.where(bits, mid, lo)
        hi = np.where(bits, hi, mid)
    # node sizes per depth: count points sharing a prefix
    leaf_depth = np.full(n, -1)
    for d in range(0, max_depth + 1):
        keys = [tuple(r) for r in paths[:, :d]]
        uniq, inv, cnt = np.unique(np.array(keys, dtype=np.int64).reshape(n, d), axis=0,
                                   return_inverse=True, return_counts=True)
        small = (cnt[inv.ravel()] <= max_batch) & (leaf_depth < 0)
        leaf_depth[small] = d
        if np.all(leaf_depth >= 0):
            break
    assert np.all(leaf_depth >= 0), "no degenerate nodes expected in this check"
    keys = [tuple(paths[p, :leaf_depth[p]]) for p in range(n)]
    order = sorted(range(n), key=lambda p: (keys[p], p))
    perm = np.array(order, dtype=np.int64)
    sizes = []
    for p in order:
        if sizes and keys[p] == keys[order[sum(sizes) - 1]] and sizes[-1] >= 0:
            sizes[-1] += 1
        else:
            sizes.append(1)
    return perm, np.concatenate([[0], np.cumsum(sizes)])


@pytest.mark.parametrize("max_batch", [20, 64, 200])
def test_octree_matches_path_brute_force(max_batch):
    rng = np.random.default_rng(max_batch)
    xyz = np.concatenate([rng.normal(size=(1500, 3)), rng.uniform(-3, 3, size=(500, 3))])
    xyz[:50] = np.round(xyz[:50], 1)            # ties with midpoints and duplicates
    perm, bp = bt.octree_batches(xyz, max_batch)
    rperm, rbp = brute_force_batches(xyz, max_batch, max_depth=20)
    assert np.array_equal(perm, rperm)
    assert np.array_equal(bp, rbp)


def test_octree_config1_partition_and_sizes():
    w = g.config_workload(1, with_density=False)
    perm, bp = bt.octree_batches(w["xyz"], 200)
    assert np.array_equal(np.sort(perm), np.arange(len(w["xyz"])))
    sizes = np.diff(bp)
    assert sizes.min() >= 1 and sizes.max() <= 200
    for b in range(len(sizes)):
        seg = perm[bp[b]:bp[b + 1]]
        assert np.all(np.diff(seg) > 0)
    perm2, bp2 = bt.octree_batches(w["xyz"], 200)
    assert np.array_equal(perm, perm2) and np.array_equal(bp, bp2)


def test_octree_degenerate_coincident_points():
    xyz = np.zeros((1000, 3)) + 1.25
    perm, bp = bt.octree_batches(xyz, 256)
    assert np.array_equal(perm, np.arange(1000))
    assert np.array_equal(bp, [0, 256, 512, 768, 1000])


def test_octree_depth_limit_chunks():
    xyz = np.zeros((301, 3))
    xyz[300] = 1.0
    perm, bp = bt.octree_batches(xyz, 256)
    # the 300 coincident points sink to depth 60 inside octant 0, then are cut in order
    assert list(np.diff(bp)) == [256, 44, 1]
    assert np.array_equal(perm, np.arange(301))


def test_octree_empty_and_single():
    perm, bp = bt.octree_batches(np.zeros((0, 3)), 10)
    assert len(perm) == 0 and list(bp) == [0]
    perm, bp = bt.octree_batches(np.ones((1, 3)), 10)
    assert list(perm) == [0] and list(bp) == [0, 1]


def test_lists_complete_and_minimal():
    w = g.config_workload(1, with_density=False)
    B = ob.Basis(w["basis"])
    xyz = w["xyz"]
    perm, bp = bt.octree_batches(xyz, 200)
    ptr, idx = bt.basis_lists(xyz, perm, bp, B)
    allphi = B.phi(xyz, np.arange(len(B.atom_xyz)))
    for b in range(len(bp) - 1):
        pts = perm[bp[b]:bp[b + 1]]
        lst = set(int(i) for i in idx[ptr[b]:ptr[b + 1]])
        nz = set(np.nonzero(np.any(allphi[pts] != 0.0, axis=0))[0].tolist())
        assert nz <= lst
        for a in set(B.fn_atom[list(lst)].tolist()):
            d = np.sqrt(((xyz[pts] - B.atom_xyz[a]) ** 2).sum(1))
            assert d.min() < B.atom_rcut[a] * (1 + 1e-12)
        assert list(idx[ptr[b]:ptr[b + 1]]) == sorted(lst)
