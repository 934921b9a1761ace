"""Grid batches and per-batch relevant-basis lists (oracle).

Section "Grid Partitioning": the integration points are split into mutually
disjoint, spatially compact batches of at most a target size ("batch size").
The paper uses a grid-adapted cut-plane method (cutplane_batches below, with the
reading stated there); the octree is the default of this build.
Reading (octree definition):

* root box = per-axis [min, max] of all points;
* a node with at most max_batch points is a leaf (a batch);
* otherwise mid = 0.5 * (lo + hi) per axis; a point goes to octant
  c = [x >= mid_x] + 2 [y >= mid_y] + 4 [z >= mid_z] (ties go high); child c
  has box [lo, mid] or [mid, hi] per axis accordingly; children are visited in
  order c = 0..7, depth-first pre-order; empty children are dropped; point
  indices stay ascending;
* degenerate node (depth >= 60, or mid equal to lo or hi on all three axes):
  its ascending index list is cut into consecutive chunks of max_batch;
* batches are numbered in emission order.

Section "Parallelization and Dimensionality Reduction": nnz(B_nu) is the set
of basis functions that are non-zero on at least one point of the batch.
Reading (relevance rule): atom A is relevant to batch b iff some point p of b
has (dx*dx + dy*dy) + dz*dz < rcA * rcA (FP64, this order, no fused
multiply-add), rcA being the largest cutoff of A's radial functions; the list
is the relevant atoms in ascending order, each expanded to its basis
functions in global order.
"""
from __future__ import annotations

import numpy as np

MAX_DEPTH = 60


def octree_batches(xyz, max_batch: int):
    """Return (perm, batch_ptr): batch b holds points perm[batch_ptr[b]:batch_ptr[b+1]]."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = len(xyz)
    leaves = []
    if n > 0:
        lo = xyz.min(axis=0)
        hi = xyz.max(axis=0)
        stack = [(np.arange(n, dtype=np.int64), lo, hi, 0)]
        while stack:
            idx, lo, hi, depth = stack.pop()
            if len(idx) <= max_batch:
                leaves.append(idx)
                continue
            mid = 0.5 * (lo + hi)
            if depth >= MAX_DEPTH or bool(np.all((mid == lo) | (mid == hi))):
                for s in range(0, len(idx), max_batch):
                    leaves.append(idx[s:s + max_batch])
                continue
            p = xyz[idx]
            octant = ((p[:, 0] >= mid[0]).astype(np.int64) + 2 * (p[:, 1] >= mid[1])
                      + 4 * (p[:, 2] >= mid[2]))
            children = []
            for c in range(8):
                sel = idx[octant == c]
                if len(sel) == 0:
                    continue
                bits = np.array([(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1], dtype=bool)
                children.append((sel, np.where(bits, mid, lo), np.where(bits, hi, mid), depth + 1))
            # pre-order: push in reverse so that octant 0 is processed first
            stack.extend(reversed(children))
    perm = np.concatenate(leaves) if leaves else np.zeros(0, dtype=np.int64)
    batch_ptr = np.zeros(len(leaves) + 1, dtype=np.int64)
    batch_ptr[1:] = np.cumsum([len(x) for x in leaves])
    return perm, batch_ptr


def cutplane_batches(xyz, max_batch: int):
    """Return (perm, batch_ptr) of the grid-adapted cut-plane partition (Section "Grid
    Partitioning": the point set is cut by planes, again and again, until every subset holds
    at most the batch size).  The paper gives no further detail; reading used here:

    * a set S with |S| <= max_batch is a batch, its indices ascending;
    * otherwise it is meant to end as k = ceil(|S| / max_batch) batches; the plane is normal
      to the axis d of largest extent max - min of S's coordinates (ties: lowest axis) and is
      placed at a quantile of the points (the grid adaptation): with S ordered by
      (coordinate d, point index) ascending, the first floor(|S| floor(k/2) / k) points form
      the lower side, the rest the upper side;
    * the lower side is processed first (depth-first pre-order); batches are numbered in
      emission order.
    Every cut splits the targeted k batches into floor(k/2) and ceil(k/2), and each side fits
    them, so every batch holds at most max_batch points and about |P| / ceil(|P| / max_batch)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = len(xyz)
    leaves = []
    stack = [np.arange(n, dtype=np.int64)] if n > 0 else []
    while stack:
        idx = stack.pop()
        m = len(idx)
        if m <= max_batch:
            leaves.append(np.sort(idx))
            continue
        k = -(-m // max_batch)
        p = xyz[idx]
        ext = p.max(axis=0) - p.min(axis=0)
        d = int(np.argmax(ext))  # first maximum: lowest axis on ties
        order = np.lexsort((idx, p[:, d]))
        n_lo = (m * (k // 2)) // k
        stack.append(idx[order[n_lo:]])
        stack.append(idx[order[:n_lo]])  # popped first
    perm = np.concatenate(leaves) if leaves else np.zeros(0, dtype=np.int64)
    batch_ptr = np.zeros(len(leaves) + 1, dtype=np.int64)
    batch_ptr[1:] = np.cumsum([len(x) for x in leaves])
    return perm, batch_ptr


def relevant_atoms_of_points(xyz_batch, atom_xyz, atom_rcut) -> np.ndarray:
    """Atoms A with some point strictly inside the sphere of radius rcA (ascending)."""
    p = np.asarray(xyz_batch, dtype=np.float64).reshape(-1, 3)
    dx = p[:, 0][:, None] - atom_xyz[None, :, 0]
    dy = p[:, 1][:, None] - atom_xyz[None, :, 1]
    dz = p[:, 2][:, None] - atom_xyz[None, :, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    rc2 = atom_rcut * atom_rcut
    return np.nonzero(np.any(d2 < rc2[None, :], axis=0))[0].astype(np.int64)


def basis_lists(xyz, perm, batch_ptr, basis):
    """Per-batch relevant-basis lists as CSR (basis_ptr int64, basis_idx int32)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    ptr = [0]
    idx = []
    for b in range(len(batch_ptr) - 1):
        pts = xyz[perm[batch_ptr[b]:batch_ptr[b + 1]]]
        atoms = relevant_atoms_of_points(pts, basis.atom_xyz, basis.atom_rcut)
        fns = basis.functions_of(atoms)
        idx.append(fns)
        ptr.append(ptr[-1] + len(fns))
    basis_idx = np.concatenate(idx).astype(np.int32) if idx else np.zeros(0, dtype=np.int32)
    return np.array(ptr, dtype=np.int64), basis_idx
