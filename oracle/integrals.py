"""Real-space quadratures on the atom-centred grid (oracle, plain FP64 numpy).

* Hamiltonian matrix, eq. (H_int_aims) restricted to a local potential:
      h_ij = sum_p w_p v_p phi_i(r_p) phi_j(r_p)
  (the operator acting on phi_j is taken to be multiplication by v_eff(r);
  the kinetic part is not part of this path).
* Overlap matrix, eq. (OverlapNoPeriodic) on the same grid: v = 1.
* Density, eq. (Density): n(r_p) = sum_ij phi_i(r_p) n_ij phi_j(r_p).  The
  density matrix is symmetric; like the symmetric matrix product the paper
  uses for it (Section "GPGPU Acceleration of the RSDD Algorithm"), only its
  upper triangle (i <= j) is read and the lower one is taken as its mirror.
* Electron count N_e = sum_p w_p n(r_p).

The point sums are split over a uniform cell grid of edge 1.5 Angstrom (at
most 4096 points per piece) purely to bound memory; every piece adds its
full contribution, restricted to the atoms with a point inside their cutoff
sphere (all others contribute exact zeros).  The cells are independent of the
octree batches.
"""
from __future__ import annotations

import numpy as np

from .batching import relevant_atoms_of_points

CELL_EDGE = 1.5
CELL_CAP = 4096


def symmetric_from_upper(D) -> np.ndarray:
    """The symmetric matrix whose upper triangle (i <= j) is that of D."""
    D = np.asarray(D, dtype=np.float64)
    U = np.triu(D)
    return U + np.triu(D, 1).T


def cell_chunks(xyz, edge: float = CELL_EDGE, cap: int = CELL_CAP):
    """Point index arrays, one per (cell, piece of at most cap points)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    if len(xyz) == 0:
        return []
    c = np.floor((xyz - xyz.min(axis=0)) / edge).astype(np.int64)
    dims = c.max(axis=0) + 1
    key = (c[:, 2] * dims[1] + c[:, 1]) * dims[0] + c[:, 0]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    cuts = np.nonzero(np.diff(ks))[0] + 1
    out = []
    for cell in np.split(order, cuts):
        for s in range(0, len(cell), cap):
            out.append(cell[s:s + cap])
    return out


def hamiltonian(basis, xyz, w, v, chunks=None) -> np.ndarray:
    """h_ij = sum_p w_p v_p phi_i(r_p) phi_j(r_p), symmetrised as (H + H^T)/2."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    wv = np.asarray(w, dtype=np.float64) * np.asarray(v, dtype=np.float64)
    H = np.zeros((basis.n_basis, basis.n_basis))
    for idx in (chunks if chunks is not None else cell_chunks(xyz)):
        atoms = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        Phi = basis.phi(xyz[idx], atoms)
        H[np.ix_(fns, fns)] += Phi.T @ (wv[idx][:, None] * Phi)
    return 0.5 * (H + H.T)


def hamiltonian_gga(basis, xyz, w, v, a, chunks=None) -> np.ndarray:
    """h_ij = sum_p w_p [v_p phi_i phi_j + a_p . (grad phi_i phi_j + phi_i grad phi_j)] at r_p,
    the local potential plus a vector field a (for a GGA, a = 2 (df/d sigma) grad n) acting on
    grad(phi_i phi_j).  Batch form of eq. batch_matrix_mult with K = Phi and
    L = (w v / 2) Phi + sum_k (w a_k) dPhi/dx_k, so that h = K^T L + L^T K (the symmetric
    rank-2k product).  a[n_points][3] in caller order."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    wv = w * np.asarray(v, dtype=np.float64)
    wa = w[:, None] * np.asarray(a, dtype=np.float64).reshape(-1, 3)
    H = np.zeros((basis.n_basis, basis.n_basis))
    for idx in (chunks if chunks is not None else cell_chunks(xyz)):
        atoms = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        Phi = basis.phi(xyz[idx], atoms)
        G = basis.grad_phi(xyz[idx], atoms)
        L = 0.5 * wv[idx][:, None] * Phi
        for k in range(3):
            L = L + wa[idx, k][:, None] * G[:, :, k]
        H[np.ix_(fns, fns)] += Phi.T @ L + L.T @ Phi
    return 0.5 * (H + H.T)


def hamiltonian_gga_entries(basis, xyz, w, v, a, pairs) -> np.ndarray:
    """hamiltonian_gga's h_ij for selected (i, j) pairs: sum over the points inside both
    cutoff spheres (sampled checks at full size)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    wv = w * np.asarray(v, dtype=np.float64)
    wa = w[:, None] * np.asarray(a, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pairs))
    for k, (i, j) in enumerate(pairs):
        fa, fb = int(basis.fn_atom[i]), int(basis.fn_atom[j])
        sel = np.ones(len(xyz), dtype=bool)
        for at in (fa, fb):
            X = basis.atom_xyz[at]
            dx = xyz[:, 0] - X[0]
            dy = xyz[:, 1] - X[1]
            dz = xyz[:, 2] - X[2]
            sel &= ((dx * dx + dy * dy) + dz * dz) < basis.atom_rcut[at] * basis.atom_rcut[at]
        idx = np.nonzero(sel)[0]
        if len(idx) == 0:
            continue
        pa = basis.phi_atom(xyz[idx], fa)[:, i - basis.atom_first[fa]]
        pb = basis.phi_atom(xyz[idx], fb)[:, j - basis.atom_first[fb]]
        ga = basis.grad_phi_atom(xyz[idx], fa)[:, i - basis.atom_first[fa], :]
        gb = basis.grad_phi_atom(xyz[idx], fb)[:, j - basis.atom_first[fb], :]
        grad_prod = ga * pb[:, None] + pa[:, None] * gb
        out[k] = float(np.sum(wv[idx] * pa * pb) + np.sum(wa[idx] * grad_prod))
    return out


def hamiltonian_ks(basis, xyz, w, v, a=None, chunks=None) -> np.ndarray:
    """h_ij = sum_p w_p [phi_i (t + v) phi_j + a_p . grad(phi_i phi_j)] at r_p, t = -1/2 lap the
    (non-relativistic) kinetic operator, symmetrised in i and j: eq. H_int_aims with h_KS
    acting on phi_j as t + v, plus the vector-field term of hamiltonian_gga (a None: none).
    Batch form of eq. batch_matrix_mult, h = K^T L + L^T K with K = Phi and
    L = (w v / 2) Phi - (w / 4) lap Phi + sum_k (w a_k) dPhi/dx_k."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    wv = w * np.asarray(v, dtype=np.float64)
    wa = None if a is None else w[:, None] * np.asarray(a, dtype=np.float64).reshape(-1, 3)
    H = np.zeros((basis.n_basis, basis.n_basis))
    for idx in (chunks if chunks is not None else cell_chunks(xyz)):
        atoms = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        Phi = basis.phi(xyz[idx], atoms)
        L = 0.5 * wv[idx][:, None] * Phi - 0.25 * w[idx][:, None] * basis.lap_phi(xyz[idx], atoms)
        if wa is not None:
            G = basis.grad_phi(xyz[idx], atoms)
            for k in range(3):
                L = L + wa[idx, k][:, None] * G[:, :, k]
        H[np.ix_(fns, fns)] += Phi.T @ L + L.T @ Phi
    return 0.5 * (H + H.T)


def kinetic(basis, xyz, w, chunks=None) -> np.ndarray:
    """t_ij = sum_p w_p (phi_i t phi_j + phi_j t phi_i) / 2: hamiltonian_ks with v = 0, no field."""
    return hamiltonian_ks(basis, xyz, w, np.zeros(len(w)), None, chunks)


def hamiltonian_ks_entries(basis, xyz, w, v, a, pairs) -> np.ndarray:
    """hamiltonian_ks's h_ij for selected (i, j) pairs (a may be None): sum over the points
    inside both cutoff spheres (sampled checks at full size)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    wv = w * np.asarray(v, dtype=np.float64)
    wa = None if a is None else w[:, None] * np.asarray(a, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pairs))
    for k, (i, j) in enumerate(pairs):
        fa, fb = int(basis.fn_atom[i]), int(basis.fn_atom[j])
        sel = np.ones(len(xyz), dtype=bool)
        for at in (fa, fb):
            X = basis.atom_xyz[at]
            dx = xyz[:, 0] - X[0]
            dy = xyz[:, 1] - X[1]
            dz = xyz[:, 2] - X[2]
            sel &= ((dx * dx + dy * dy) + dz * dz) < basis.atom_rcut[at] * basis.atom_rcut[at]
        idx = np.nonzero(sel)[0]
        if len(idx) == 0:
            continue
        ia, jb = i - basis.atom_first[fa], j - basis.atom_first[fb]
        pa = basis.phi_atom(xyz[idx], fa)[:, ia]
        pb = basis.phi_atom(xyz[idx], fb)[:, jb]
        la = basis.lap_phi_atom(xyz[idx], fa)[:, ia]
        lb = basis.lap_phi_atom(xyz[idx], fb)[:, jb]
        val = np.sum(wv[idx] * pa * pb) - 0.25 * np.sum(w[idx] * (pa * lb + la * pb))
        if wa is not None:
            ga = basis.grad_phi_atom(xyz[idx], fa)[:, ia, :]
            gb = basis.grad_phi_atom(xyz[idx], fb)[:, jb, :]
            val += np.sum(wa[idx] * (ga * pb[:, None] + pa[:, None] * gb))
        out[k] = float(val)
    return out


def overlap(basis, xyz, w, chunks=None) -> np.ndarray:
    """s_ij on the grid: the v = 1 case of the Hamiltonian quadrature."""
    return hamiltonian(basis, xyz, w, np.ones(len(w)), chunks)


def density(basis, xyz, D, chunks=None) -> np.ndarray:
    """n(r_p) = sum_ij phi_i(r_p) D_ij phi_j(r_p) for every point (caller order)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    Ds = symmetric_from_upper(D)
    n = np.zeros(len(xyz))
    for idx in (chunks if chunks is not None else cell_chunks(xyz)):
        atoms = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        Phi = basis.phi(xyz[idx], atoms)
        T = Phi @ Ds[np.ix_(fns, fns)]
        n[idx] = (T * Phi).sum(axis=1)
    return n


def density_gradient(basis, xyz, D, chunks=None):
    """(n, grad n) at every point: grad n(r_p) = 2 sum_ij grad phi_i(r_p) D_ij phi_j(r_p) for
    symmetric D (the gradient of eq. Density that the paper names beside it and in the
    subsection "Density and Density Derivatives, Force and Stress Tensor Components"):
    T = Phi D, n = rowsum(T * Phi), grad n = 2 rowsum(T * grad Phi) per component."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    Ds = symmetric_from_upper(D)
    n = np.zeros(len(xyz))
    g = np.zeros((len(xyz), 3))
    for idx in (chunks if chunks is not None else cell_chunks(xyz)):
        atoms = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        Phi = basis.phi(xyz[idx], atoms)
        G = basis.grad_phi(xyz[idx], atoms)
        T = Phi @ Ds[np.ix_(fns, fns)]
        n[idx] = (T * Phi).sum(axis=1)
        for k in range(3):
            g[idx, k] = 2.0 * (T * G[:, :, k]).sum(axis=1)
    return n, g


def density_gradient_at(basis, pts, D) -> np.ndarray:
    """grad n at selected points, one point at a time (sampled checks at full size)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    Ds = symmetric_from_upper(D)
    out = np.zeros((len(pts), 3))
    for k, p in enumerate(pts):
        atoms = relevant_atoms_of_points(p[None, :], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        phi = basis.phi(p[None, :], atoms)[0]
        G = basis.grad_phi(p[None, :], atoms)[0]
        out[k] = 2.0 * (G.T @ (Ds[np.ix_(fns, fns)] @ phi))
    return out


def pulay_forces(basis, xyz, w, v, D, Q, chunks=None, kinetic=True) -> np.ndarray:
    """Local Pulay forces F_A [n_atoms][3], the density-only part of the Pulay force that follows
    eq. forces:
        F_A = -2 sum_ij sum_p w_p [grad_A phi_i](r_p) (n_ij [h_KS phi_j](r_p) - q_ij phi_j(r_p)),
    h_KS = t + v with t = -1/2 lap the (non-relativistic) kinetic operator and v the local
    potential (kinetic=False: v alone), n the density matrix D and q the energy-weighted density
    matrix Q (eq. E_Weighted_DM), both symmetric, upper triangles read.  grad_A phi_i = -grad
    phi_i for the functions i centred on A and 0 for all others, so with, per point,
        M = w ((v Phi - lap Phi / 2) D - Phi Q),
        f_i = sum_p grad phi_i(r_p) M_pi,   F_A = 2 sum_{i on A} f_i."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    Ds = symmetric_from_upper(D)
    Qs = symmetric_from_upper(Q)
    f = np.zeros((basis.n_basis, 3))
    for idx in (chunks if chunks is not None else cell_chunks(xyz)):
        atoms = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        Phi = basis.phi(xyz[idx], atoms)
        G = basis.grad_phi(xyz[idx], atoms)
        hPhi = v[idx][:, None] * Phi  # h_KS phi_j at the points
        if kinetic:
            hPhi = hPhi - 0.5 * basis.lap_phi(xyz[idx], atoms)
        M = w[idx][:, None] * (hPhi @ Ds[np.ix_(fns, fns)] - Phi @ Qs[np.ix_(fns, fns)])
        for k in range(3):
            f[fns, k] += (G[:, :, k] * M).sum(axis=0)
    F = np.zeros((len(basis.atom_xyz), 3))
    for a in range(len(basis.atom_xyz)):
        F[a] = 2.0 * f[basis.atom_first[a]:basis.atom_first[a + 1]].sum(axis=0)
    return F


def pulay_forces_at(basis, xyz, w, v, D, Q, atoms, kinetic=True) -> np.ndarray:
    """pulay_forces for selected atoms only: the points inside atom A's cutoff sphere (the
    only ones where grad_A phi is not zero), against every function reaching them (sampled
    checks at full size)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    Ds = symmetric_from_upper(D)
    Qs = symmetric_from_upper(Q)
    out = np.zeros((len(atoms), 3))
    for k, A in enumerate(atoms):
        A = int(A)
        X = basis.atom_xyz[A]
        dx = xyz[:, 0] - X[0]
        dy = xyz[:, 1] - X[1]
        dz = xyz[:, 2] - X[2]
        sel = np.nonzero(((dx * dx + dy * dy) + dz * dz) < basis.atom_rcut[A] * basis.atom_rcut[A])[0]
        fa = np.arange(basis.atom_first[A], basis.atom_first[A + 1])
        for piece in cell_chunks(xyz[sel]):
            idx = sel[piece]
            rel = relevant_atoms_of_points(xyz[idx], basis.atom_xyz, basis.atom_rcut)
            fns = basis.functions_of(rel)
            Phi = basis.phi(xyz[idx], rel)
            hPhi = v[idx][:, None] * Phi
            if kinetic:
                hPhi = hPhi - 0.5 * basis.lap_phi(xyz[idx], rel)
            GA = basis.grad_phi_atom(xyz[idx], A)
            M = w[idx][:, None] * (hPhi @ Ds[np.ix_(fns, fa)] - Phi @ Qs[np.ix_(fns, fa)])
            for c in range(3):
                out[k, c] += 2.0 * float((GA[:, :, c] * M).sum())
    return out


def electron_count(w, n) -> float:
    """N_e = sum_p w_p n(r_p)."""
    return float(np.dot(np.asarray(w, dtype=np.float64), np.asarray(n, dtype=np.float64)))


def density_at(basis, pts, D) -> np.ndarray:
    """n at selected points, one point at a time (sampled checks at full size)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    Ds = symmetric_from_upper(D)
    out = np.zeros(len(pts))
    for k, p in enumerate(pts):
        atoms = relevant_atoms_of_points(p[None, :], basis.atom_xyz, basis.atom_rcut)
        if len(atoms) == 0:
            continue
        fns = basis.functions_of(atoms)
        phi = basis.phi(p[None, :], atoms)[0]
        out[k] = phi @ Ds[np.ix_(fns, fns)] @ phi
    return out


def hamiltonian_entries(basis, xyz, w, v, pairs) -> np.ndarray:
    """h_ij for selected (i, j) pairs: sum over the points inside both cutoff spheres."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    wv = np.asarray(w, dtype=np.float64) * np.asarray(v, dtype=np.float64)
    out = np.zeros(len(pairs))
    for k, (i, j) in enumerate(pairs):
        a, b = int(basis.fn_atom[i]), int(basis.fn_atom[j])
        sel = np.ones(len(xyz), dtype=bool)
        for at in (a, b):
            X = basis.atom_xyz[at]
            dx = xyz[:, 0] - X[0]
            dy = xyz[:, 1] - X[1]
            dz = xyz[:, 2] - X[2]
            sel &= ((dx * dx + dy * dy) + dz * dz) < basis.atom_rcut[at] * basis.atom_rcut[at]
        idx = np.nonzero(sel)[0]
        if len(idx) == 0:
            continue
        pa = basis.phi_atom(xyz[idx], a)[:, i - basis.atom_first[a]]
        pb = basis.phi_atom(xyz[idx], b)[:, j - basis.atom_first[b]]
        out[k] = float(np.sum(wv[idx] * pa * pb))
    return out


def hamiltonian_batched(basis, xyz, w, v, perm, batch_ptr, basis_ptr, basis_idx) -> np.ndarray:
    """eq. (H_decomp)/(H_contrib_batch): h = sum over batches of the dense batch matrices
    K L (eq. batch_matrix_mult) restricted to each batch's list, then symmetrised."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    wv = np.asarray(w, dtype=np.float64) * np.asarray(v, dtype=np.float64)
    H = np.zeros((basis.n_basis, basis.n_basis))
    for b in range(len(batch_ptr) - 1):
        idx = perm[batch_ptr[b]:batch_ptr[b + 1]]
        fns = np.asarray(basis_idx[basis_ptr[b]:basis_ptr[b + 1]], dtype=np.int64)
        if len(fns) == 0:
            continue
        atoms = np.unique(basis.fn_atom[fns])
        Phi = basis.phi(xyz[idx], atoms)
        K = (wv[idx][:, None] * Phi).T
        H[np.ix_(fns, fns)] += K @ Phi
    return 0.5 * (H + H.T)


def density_batched(basis, xyz, D, perm, batch_ptr, basis_ptr, basis_idx) -> np.ndarray:
    """n per batch through the batch density matrix n_ij[B] (Section "GPGPU Acceleration of
    the RSDD Algorithm": reduce the full density matrix to the batch's list, then a matrix
    product and a row-wise dot product)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    Ds = symmetric_from_upper(D)
    n = np.zeros(len(xyz))
    for b in range(len(batch_ptr) - 1):
        idx = perm[batch_ptr[b]:batch_ptr[b + 1]]
        fns = np.asarray(basis_idx[basis_ptr[b]:basis_ptr[b + 1]], dtype=np.int64)
        if len(fns) == 0:
            continue
        atoms = np.unique(basis.fn_atom[fns])
        Phi = basis.phi(xyz[idx], atoms)
        n[idx] = ((Phi @ Ds[np.ix_(fns, fns)]) * Phi).sum(axis=1)
    return n


def batch_phi(basis, xyz, perm, batch_ptr, basis_ptr, basis_idx, b) -> np.ndarray:
    """The dense batch basis matrix [|B|, m] (point-major) of batch b."""
    idx = perm[batch_ptr[b]:batch_ptr[b + 1]]
    fns = np.asarray(basis_idx[basis_ptr[b]:basis_ptr[b + 1]], dtype=np.int64)
    atoms = np.unique(basis.fn_atom[fns]) if len(fns) else []
    return basis.phi(np.asarray(xyz, dtype=np.float64).reshape(-1, 3)[idx], atoms)
