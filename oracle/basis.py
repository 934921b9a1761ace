"""Atom-centred numeric basis functions evaluated at grid points (oracle).

phi_i(r) = R_{s(i)}(|r - R_A|) * Y_{l(i) m(i)}(unit(r - R_A)) for the basis
function i centred on atom A, the basis of eq. (EVNonPeriodic).  The radial
parts vanish beyond the confining radius (Section "Computational Choices in
FHI-aims"); reading used here: phi_i(r) = 0 exactly when
(dx*dx + dy*dy) + dz*dz >= rcut_s * rcut_s, evaluated in that order in FP64, the
same test that decides batch relevance.  At |r - R_A| = 0 the direction is
taken as (0, 0, 1).

Global basis order: atom-major, then the species' shell order, then m = -l..l.

Gradient (for the density gradient the paper names beside eq. (Density)): with
u = (r - R_A)/|r - R_A| and G = dY/du (the harmonic polynomial differentiated in
the components of u), grad phi = R'(r) u Y + (R/r) (G - u (u . G)), the chain
rule through du/dr = (I - u u^T)/r.  Reading: grad phi = 0 where phi is zero by
the cutoff test and for |r - R_A| <= rmin (the clamped, constant part of the
spline).

Laplacian (for the kinetic term -1/2 lap of the Hamiltonian): Y_lm is a spherical
harmonic of degree l, so lap phi = (R'' + 2 R'/r - l(l+1) R/r^2) Y_lm(u), with the
radial factor from the spline (oracle.spline.radial_laplacian); zero where grad phi
is zero by the reading above.
"""
from __future__ import annotations

import numpy as np

from .spline import RadialSpline, evaluate_t, spline_t
from .ylm import real_ylm, real_ylm_grad


class Basis:
    """Basis description (the same fields as the library's basis descriptor)."""

    def __init__(self, desc):
        self.atom_xyz = np.asarray(desc["atom_xyz"], dtype=np.float64).reshape(-1, 3)
        self.atom_species = np.asarray(desc["atom_species"], dtype=np.int64)
        ptr = np.asarray(desc["species_shell_ptr"], dtype=np.int64)
        shell_l = np.asarray(desc["shell_l"], dtype=np.int64)
        shell_rad = np.asarray(desc["shell_radial"], dtype=np.int64)
        rmin = np.asarray(desc["radial_rmin"], dtype=np.float64)
        rcut = np.asarray(desc["radial_rcut"], dtype=np.float64)
        samples = np.asarray(desc["radial_samples"], dtype=np.float64)
        self.splines = [RadialSpline(samples[k], rmin[k], rcut[k]) for k in range(len(rmin))]
        fn_atom, fn_rad, fn_l, fn_lm = [], [], [], []
        self.atom_first = np.zeros(len(self.atom_xyz) + 1, dtype=np.int64)
        self.atom_rcut = np.zeros(len(self.atom_xyz))
        for a, s in enumerate(self.atom_species):
            self.atom_first[a] = len(fn_atom)
            rc = 0.0
            for j in range(ptr[s], ptr[s + 1]):
                l = int(shell_l[j])
                rc = max(rc, rcut[shell_rad[j]])
                for m in range(-l, l + 1):
                    fn_atom.append(a)
                    fn_rad.append(int(shell_rad[j]))
                    fn_l.append(l)
                    fn_lm.append(l * l + m + l)
            self.atom_rcut[a] = rc
        self.atom_first[-1] = len(fn_atom)
        self.fn_atom = np.array(fn_atom, dtype=np.int64)
        self.fn_radial = np.array(fn_rad, dtype=np.int64)
        self.fn_l = np.array(fn_l, dtype=np.int64)
        self.fn_lm = np.array(fn_lm, dtype=np.int64)
        self.n_basis = len(fn_atom)

    def functions_of(self, atoms) -> np.ndarray:
        """Global indices of the basis functions of the given atoms (ascending atoms)."""
        atoms = np.asarray(atoms, dtype=np.int64)
        if len(atoms) == 0:
            return np.zeros(0, dtype=np.int64)
        return np.concatenate([np.arange(self.atom_first[a], self.atom_first[a + 1]) for a in atoms])

    def phi_atom(self, pts, a) -> np.ndarray:
        """phi of every basis function of atom a at pts[n, 3] -> [n, nfn(a)]."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        X = self.atom_xyz[a]
        dx = pts[:, 0] - X[0]
        dy = pts[:, 1] - X[1]
        dz = pts[:, 2] - X[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        r = np.sqrt(d2)
        safe = np.where(r > 0.0, r, 1.0)
        u = np.stack([np.where(r > 0.0, dx / safe, 0.0), np.where(r > 0.0, dy / safe, 0.0),
                      np.where(r > 0.0, dz / safe, 1.0)], axis=1)
        Y = real_ylm(u)
        fns = range(self.atom_first[a], self.atom_first[a + 1])
        out = np.zeros((len(pts), len(fns)))
        for c, i in enumerate(fns):
            sp = self.splines[self.fn_radial[i]]
            inside = d2 < sp.rcut * sp.rcut
            R = evaluate_t(spline_t(r, sp.rmin, sp.rcut, sp.n), sp.y, sp.M)
            out[:, c] = np.where(inside, R * Y[:, self.fn_lm[i]], 0.0)
        return out

    def grad_phi_atom(self, pts, a) -> np.ndarray:
        """grad phi of every basis function of atom a at pts[n, 3] -> [n, nfn(a), 3]."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        X = self.atom_xyz[a]
        dx = pts[:, 0] - X[0]
        dy = pts[:, 1] - X[1]
        dz = pts[:, 2] - X[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        r = np.sqrt(d2)
        safe = np.where(r > 0.0, r, 1.0)
        u = np.stack([np.where(r > 0.0, dx / safe, 0.0), np.where(r > 0.0, dy / safe, 0.0),
                      np.where(r > 0.0, dz / safe, 1.0)], axis=1)
        Y = real_ylm(u)
        G = real_ylm_grad(u)                                  # [n, 16, 3]
        Gt = G - u[:, None, :] * np.einsum("nlk,nk->nl", G, u)[:, :, None]  # tangential part
        fns = range(self.atom_first[a], self.atom_first[a + 1])
        out = np.zeros((len(pts), len(fns), 3))
        for c, i in enumerate(fns):
            sp = self.splines[self.fn_radial[i]]
            ok = (d2 < sp.rcut * sp.rcut) & (r > sp.rmin)
            R = evaluate_t(spline_t(r, sp.rmin, sp.rcut, sp.n), sp.y, sp.M)
            dR = sp.deriv_at_r(r)
            lm = self.fn_lm[i]
            g = dR[:, None] * u * Y[:, lm][:, None] + (R / safe)[:, None] * Gt[:, lm, :]
            out[:, c, :] = np.where(ok[:, None], g, 0.0)
        return out

    def lap_phi_atom(self, pts, a) -> np.ndarray:
        """Laplacian of every basis function of atom a at pts[n, 3] -> [n, nfn(a)]."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        X = self.atom_xyz[a]
        dx = pts[:, 0] - X[0]
        dy = pts[:, 1] - X[1]
        dz = pts[:, 2] - X[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        r = np.sqrt(d2)
        safe = np.where(r > 0.0, r, 1.0)
        u = np.stack([np.where(r > 0.0, dx / safe, 0.0), np.where(r > 0.0, dy / safe, 0.0),
                      np.where(r > 0.0, dz / safe, 1.0)], axis=1)
        Y = real_ylm(u)
        fns = range(self.atom_first[a], self.atom_first[a + 1])
        out = np.zeros((len(pts), len(fns)))
        for c, i in enumerate(fns):
            sp = self.splines[self.fn_radial[i]]
            ok = (d2 < sp.rcut * sp.rcut) & (r > sp.rmin)
            lap = sp.laplacian_at_r(r, int(self.fn_l[i]))
            out[:, c] = np.where(ok, lap * Y[:, self.fn_lm[i]], 0.0)
        return out

    def lap_phi(self, pts, atoms) -> np.ndarray:
        """Laplacian of the functions of `atoms` (ascending) at pts -> [n, m]."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        if len(atoms) == 0:
            return np.zeros((len(pts), 0))
        return np.concatenate([self.lap_phi_atom(pts, a) for a in atoms], axis=1)

    def grad_phi(self, pts, atoms) -> np.ndarray:
        """grad phi of the functions of `atoms` (ascending) at pts -> [n, m, 3]."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        if len(atoms) == 0:
            return np.zeros((len(pts), 0, 3))
        return np.concatenate([self.grad_phi_atom(pts, a) for a in atoms], axis=1)

    def phi(self, pts, atoms) -> np.ndarray:
        """phi of the functions of `atoms` (ascending) at pts -> [n, m] in global order."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        if len(atoms) == 0:
            return np.zeros((len(pts), 0))
        return np.concatenate([self.phi_atom(pts, a) for a in atoms], axis=1)

    def relevant_atoms(self, pts) -> np.ndarray:
        """Atoms with at least one point strictly inside their cutoff sphere (ascending)."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        out = []
        for a in range(len(self.atom_xyz)):
            X = self.atom_xyz[a]
            dx = pts[:, 0] - X[0]
            dy = pts[:, 1] - X[1]
            dz = pts[:, 2] - X[2]
            d2 = (dx * dx + dy * dy) + dz * dz
            if np.any(d2 < self.atom_rcut[a] * self.atom_rcut[a]):
                out.append(a)
        return np.array(out, dtype=np.int64)
