"""Pins of the oracle's cut-plane batcher: a hand-worked split of points on a line, two
separated clusters that must come out as the clusters, and the invariants every partition has
(disjoint cover, batch size bound, the batch count the quantile cuts give, ascending indices)."""
import numpy as np
import pytest

from oracle import batching as ob
from workloads import config_workload


def batches(perm, bp):
    return [list(perm[bp[b]:bp[b + 1]]) for b in range(len(bp) - 1)]


def test_worked_example_on_a_line():
    # 10 points x = 0..9 (shuffled indices), max 3: k = 4 -> 5 | 5; each 5 -> k = 2 -> 2 | 3
    xs = np.array([7, 2, 9, 0, 4, 1, 8, 3, 6, 5], dtype=np.float64)
    xyz = np.stack([xs, np.zeros(10), np.zeros(10)], axis=1)
    perm, bp = ob.cutplane_batches(xyz, 3)
    got = [sorted(xs[b].tolist()) for b in batches(perm, bp)]
    assert got == [[0.0, 1.0], [2.0, 3.0, 4.0], [5.0, 6.0], [7.0, 8.0, 9.0]]
    assert all(b == sorted(b) for b in batches(perm, bp))


def test_ties_split_by_index_and_longest_axis():
    # all x equal, y spread wider than z: the cut is along y
    xyz = np.array([[1.0, 0.0, 0.0], [1.0, 3.0, 0.1], [1.0, 1.0, 0.2], [1.0, 2.0, 0.0]])
    perm, bp = ob.cutplane_batches(xyz, 2)
    assert batches(perm, bp) == [[0, 2], [1, 3]]
    # identical points: the order by index decides
    perm, bp = ob.cutplane_batches(np.zeros((5, 3)), 2)
    assert batches(perm, bp) == [[0], [1, 2], [3, 4]]


def test_separated_clusters_are_batches():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(50, 3))
    b = rng.normal(size=(50, 3)) + np.array([20.0, 0.0, 0.0])
    xyz = np.concatenate([b, a])[rng.permutation(100)]
    perm, bp = ob.cutplane_batches(xyz, 50)
    bs = batches(perm, bp)
    assert len(bs) == 2
    assert {tuple(np.sign(xyz[bb, 0] - 10.0).astype(int)) for bb in map(np.array, bs)} == {(-1,) * 50, (1,) * 50}


@pytest.mark.parametrize("mb", [100, 200, 256])
def test_invariants_on_a_workload(mb):
    xyz = config_workload(1)["xyz"]
    perm, bp = ob.cutplane_batches(xyz, mb)
    assert np.array_equal(np.sort(perm), np.arange(len(xyz)))
    sizes = np.diff(bp)
    assert sizes.max() <= mb and sizes.min() >= 1
    assert len(sizes) == -(-len(xyz) // mb)  # quantile cuts give exactly ceil(n / mb) batches
    for b in batches(perm, bp):
        assert b == sorted(b)


def test_planted_midpoint_cut_fails_the_worked_example():
    """Cutting at the geometric midpoint instead of the point quantile changes the batches of
    the worked example (points clustered towards one end)."""
    xs = np.array([0.0, 0.1, 0.2, 0.3, 0.4, 9.0])
    xyz = np.stack([xs, np.zeros(6), np.zeros(6)], axis=1)
    perm, bp = ob.cutplane_batches(xyz, 3)
    assert batches(perm, bp) == [[0, 1, 2], [3, 4, 5]]
    mid = 0.5 * (xs.min() + xs.max())
    assert [list(np.nonzero(xs < mid)[0]), list(np.nonzero(xs >= mid)[0])] != batches(perm, bp)
