"""Seeded synthetic inputs for the real-space grid operations.

This module builds inputs only: atom geometries, per-species shells, sampled
radial functions, atom-centred integration grids with partition weights, a
potential sampled at the points and a density matrix.  It holds none of the
arithmetic of the integration method (splines, spherical harmonics, batching,
relevance lists and the contractions live in the oracle and in the HIP
library, separately).  Both sides consume what this module produces.

The paper's own workloads (FHI-aims "tight" species, bulk supercells, the
Bi2Se3 slab) are not available; these inputs stand in for their shapes:
atom-centred shell grids (Section "Real-Space Integration Grids"), confined
numeric radial functions (Section "Computational Choices in FHI-aims"),
partition-of-unity weights (Becke) and D = C C^T (eq. DM_from_EV with f = 1).

Every random draw comes from
    numpy.random.default_rng(SeedSequence([cfg, structure, stream, iteration]))
with streams 0 geometry, 1 radial functions, 2 potential, 3 density matrix,
4 arrivals and choices.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

STREAM_GEOMETRY, STREAM_RADIAL, STREAM_POTENTIAL, STREAM_DENSITY, STREAM_ARRIVAL, STREAM_ENERGY = range(6)

N_KNOTS = 200
R_MIN = 1.0e-4
R_M = 1.0  # radial-grid scale (Angstrom)

# Per-configuration shapes (sizes in Angstrom).
CONFIGS = {
    1: dict(shells=(0, 0, 1), rcut=4.0, n_r=30, n_ang=110, max_batch=200, n_gauss=8, n_occ=4,
            d_max=None),
    2: dict(shells=(0, 0, 0, 1, 1, 2), rcut=5.0, n_r=50, n_ang=302, max_batch=256, n_gauss=64,
            n_occ=200, d_max=10.0),
    3: dict(shells=(0, 0, 0, 1, 1, 2), rcut=5.0, n_r=50, n_ang=302, max_batch=256, n_gauss=64,
            n_occ=None, d_max=10.0),
    4: dict(shells=(0, 0, 1, 1, 1, 2, 2, 3), rcut=6.0, n_r=60, n_ang=434, max_batch=256,
            n_gauss=256, n_occ=1500, d_max=12.0),
}
CONFIG3_N_STRUCTURES = 64


def rng_for(cfg: int, structure: int, stream: int, iteration: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, structure, stream, iteration]))


# ----------------------------------------------------------------------------------------------
# native helper (partition weights, Gaussian sum)

_LIB = None
_LIB_LOCK = threading.Lock()
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gridgen.c")
_SO = os.path.join(_HERE, "_gridgen.so")


def build_native(force: bool = False) -> str:
    """Compile gridgen.c with gcc/OpenMP into _gridgen.so (in place)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    with _LIB_LOCK:
        if _LIB is None:
            lib = ctypes.CDLL(build_native())
            d = ctypes.POINTER(ctypes.c_double)
            lib.gg_becke_owner_weight.argtypes = [ctypes.c_int64, d, ctypes.c_double, ctypes.c_int64,
                                                  d, ctypes.POINTER(ctypes.c_int32), d]
            lib.gg_becke_owner_weight.restype = ctypes.c_int
            lib.gg_gaussian_sum.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, d]
            lib.gg_gaussian_sum.restype = None
            _LIB = lib
    return _LIB


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------------------------
# geometries

def geometry_random_cube(n_atoms: int, side: float, min_sep: float, rng) -> np.ndarray:
    """Sequential rejection sampling of U([0, side]^3) with a minimum separation."""
    out = []
    while len(out) < n_atoms:
        p = rng.uniform(0.0, side, size=3)
        if all(np.sqrt(((p - q) ** 2).sum()) >= min_sep for q in out):
            out.append(p)
    return np.array(out, dtype=np.float64)


def geometry_cubic_block(nx: int, ny: int, nz: int, a: float, sigma: float, rng) -> np.ndarray:
    """Sites (i, j, k) * a with i fastest, plus N(0, sigma^2) jitter."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sites = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * a
    return sites + rng.normal(0.0, sigma, size=sites.shape)


def geometry_sc_first_n(n: int, a: float, sigma: float, rng) -> np.ndarray:
    """First n sites (i fastest) of a ceil(n^(1/3))^3 simple-cubic lattice, jittered."""
    s = 1
    while s ** 3 < n:
        s += 1
    k, j, i = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    sites = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)[:n].astype(np.float64) * a
    return sites + rng.normal(0.0, sigma, size=sites.shape)


def geometry_layered_slab(per_layer: int, n_layers: int, window: float, rng, nn: float = 2.5,
                          layer_dz: float = 3.75, shift: float = 2.5, sigma: float = 0.05):
    """Honeycomb layers (nearest neighbour nn) in a square window, stacked along z.

    Rectangular cell sqrt(3)*nn x 3*nn with sites (0,0), (ax/2, nn/2), (ax/2, 3nn/2), (0, 2nn);
    sites inside [0, window)^2, keep the per_layer nearest the window centre (stable order),
    layers at z = layer_dz * l, odd layers shifted by +shift in x, then N(0, sigma^2) jitter.
    """
    ax, ay = math.sqrt(3.0) * nn, 3.0 * nn
    basis = np.array([[0.0, 0.0], [ax / 2, nn / 2], [ax / 2, 1.5 * nn], [0.0, 2.0 * nn]])
    sites = []
    for cy in range(int(window / ay) + 2):
        for cx in range(int(window / ax) + 2):
            for b in basis:
                x, y = cx * ax + b[0], cy * ay + b[1]
                if 0.0 <= x < window and 0.0 <= y < window:
                    sites.append((x, y))
    sites = np.array(sites, dtype=np.float64)
    c = window / 2.0
    d2 = (sites[:, 0] - c) ** 2 + (sites[:, 1] - c) ** 2
    order = np.argsort(d2, kind="stable")[:per_layer]
    plane = sites[order]
    layers = []
    for l in range(n_layers):
        xy = plane.copy()
        if l % 2 == 1:
            xy[:, 0] += shift
        layers.append(np.column_stack([xy, np.full(len(xy), layer_dz * l)]))
    xyz = np.concatenate(layers, axis=0)
    return xyz + rng.normal(0.0, sigma, size=xyz.shape)


# ----------------------------------------------------------------------------------------------
# radial functions and basis description

def knot_radii(rmin: float, rcut: float, n_knots: int) -> np.ndarray:
    """Logarithmic knots r_k = rmin * (rcut/rmin)^(k/(N-1)); the last one is rcut exactly."""
    k = np.arange(n_knots, dtype=np.float64)
    r = rmin * np.exp(k * (math.log(rcut / rmin) / (n_knots - 1)))
    r[0] = rmin
    r[-1] = rcut
    return r


_GL4000 = None


def _gauss_legendre_4000():
    global _GL4000
    if _GL4000 is None:
        _GL4000 = np.polynomial.legendre.leggauss(4000)
    return _GL4000


def synthetic_radial(l: int, rcut: float, rng, r: np.ndarray) -> np.ndarray:
    """R(r) = f_c(r) r^l sum_g c_g exp(-alpha_g r^2), f_c = (1-(r/rcut)^2)^3, normalised so that
    int_0^rcut R^2 r^2 dr = 1 (4000-point Gauss-Legendre)."""
    cg = rng.normal(0.0, 1.0, size=3)
    ag = np.exp(rng.uniform(math.log(0.25), math.log(4.0), size=3))

    def R(x):
        x = np.asarray(x, dtype=np.float64)
        fc = np.where(x < rcut, (1.0 - (x / rcut) ** 2) ** 3, 0.0)
        return fc * x ** l * (cg[None, :] * np.exp(-ag[None, :] * x[:, None] ** 2)).sum(axis=1)

    xg, wg = _gauss_legendre_4000()
    xr = 0.5 * rcut * (xg + 1.0)
    norm = math.sqrt(float((0.5 * rcut * wg * R(xr) ** 2 * xr ** 2).sum()))
    y = R(r) / norm
    y[r >= rcut] = 0.0
    return y


def make_basis(atom_xyz, species_of_atom, species_shells, species_rcut, cfg, structure,
               n_knots=N_KNOTS, rmin=R_MIN):
    """Basis description with one radial function per (species, shell)."""
    rng = rng_for(cfg, structure, STREAM_RADIAL)
    shell_ptr = [0]
    shell_l, shell_radial, rrmin, rrcut, samples = [], [], [], [], []
    for s, shells in enumerate(species_shells):
        rc = float(species_rcut[s])
        r = knot_radii(rmin, rc, n_knots)
        for l in shells:
            shell_l.append(int(l))
            shell_radial.append(len(samples))
            rrmin.append(rmin)
            rrcut.append(rc)
            samples.append(synthetic_radial(int(l), rc, rng, r))
        shell_ptr.append(len(shell_l))
    return dict(
        atom_xyz=np.ascontiguousarray(atom_xyz, dtype=np.float64),
        atom_species=np.ascontiguousarray(species_of_atom, dtype=np.int32),
        species_shell_ptr=np.array(shell_ptr, dtype=np.int32),
        shell_l=np.array(shell_l, dtype=np.int32),
        shell_radial=np.array(shell_radial, dtype=np.int32),
        radial_rmin=np.array(rrmin, dtype=np.float64),
        radial_rcut=np.array(rrcut, dtype=np.float64),
        radial_samples=np.ascontiguousarray(np.array(samples, dtype=np.float64)),
        n_knots=int(n_knots),
    )


def atom_rcut(basis) -> np.ndarray:
    """Largest radial cutoff of each atom's species."""
    out = np.zeros(len(basis["atom_species"]))
    for a, s in enumerate(basis["atom_species"]):
        sh = range(basis["species_shell_ptr"][s], basis["species_shell_ptr"][s + 1])
        out[a] = max(basis["radial_rcut"][basis["shell_radial"][j]] for j in sh)
    return out


def basis_atom_index(basis) -> np.ndarray:
    """Owning atom of every basis function (atom-major, shell order, m = -l..l)."""
    out = []
    for a, s in enumerate(basis["atom_species"]):
        for j in range(basis["species_shell_ptr"][s], basis["species_shell_ptr"][s + 1]):
            out += [a] * (2 * int(basis["shell_l"][j]) + 1)
    return np.array(out, dtype=np.int64)


def n_basis(basis) -> int:
    return int(len(basis_atom_index(basis)))


# ----------------------------------------------------------------------------------------------
# grids, weights, potential, density matrix

def radial_grid(n_r: int, r_m: float = R_M):
    """Becke's Gauss-Chebyshev (second kind) map: x_i = cos(i pi/(n+1)), r = r_m (1+x)/(1-x),
    weights include r^2 dr/dx."""
    i = np.arange(1, n_r + 1, dtype=np.float64)
    th = i * math.pi / (n_r + 1)
    x = np.cos(th)
    r = r_m * (1.0 + x) / (1.0 - x)
    w = (math.pi / (n_r + 1)) * np.sin(th) * 2.0 * r_m / (1.0 - x) ** 2 * r ** 2
    return r, w


def fibonacci_sphere(n: int):
    """Spherical Fibonacci directions z_k = 1-(2k+1)/n, phi_k = k pi (3 - sqrt 5); weight 4 pi/n."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    ph = k * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1), np.full(n, 4.0 * math.pi / n)


def becke_owner_weight(atom_xyz, rp, pts, owner) -> np.ndarray:
    out = np.empty(len(pts))
    atom_xyz = np.ascontiguousarray(atom_xyz, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    owner = np.ascontiguousarray(owner, dtype=np.int32)
    rc = _lib().gg_becke_owner_weight(len(atom_xyz), _dptr(atom_xyz), float(rp), len(pts), _dptr(pts),
                                      owner.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(out))
    if rc != 0:
        raise RuntimeError("partition weights failed (%d)" % rc)
    return out


def becke_owner_weight_numpy(atom_xyz, rp, pts, owner) -> np.ndarray:
    """Slow reference of becke_owner_weight, for tests on small inputs."""
    out = np.zeros(len(pts))
    for p, r in enumerate(pts):
        d = np.sqrt(((r[None, :] - atom_xyz) ** 2).sum(axis=1))
        nb = np.nonzero(d < rp)[0]
        if owner[p] not in nb:
            continue
        P = np.ones(len(nb))
        for ii, b in enumerate(nb):
            for c in nb:
                if c == b:
                    continue
                mu = (d[b] - d[c]) / math.sqrt(((atom_xyz[b] - atom_xyz[c]) ** 2).sum())
                for _ in range(3):
                    mu = 1.5 * mu - 0.5 * mu ** 3
                P[ii] *= 0.5 * (1.0 - mu)
        s = P.sum()
        out[p] = P[list(nb).index(owner[p])] / s if s > 0 else 0.0
    return out


def make_grid(atom_xyz, rp, n_r, n_ang):
    """Atom-centred shell grid; point p = (A n_r + i) n_ang + k.  Returns xyz, w, owner."""
    atom_xyz = np.asarray(atom_xyz, dtype=np.float64)
    r, wr = radial_grid(n_r)
    u, wa = fibonacci_sphere(n_ang)
    shell = (r[:, None, None] * u[None, :, :]).reshape(-1, 3)       # [n_r*n_ang, 3]
    wsh = (wr[:, None] * wa[None, :]).reshape(-1)
    n_at = len(atom_xyz)
    xyz = (atom_xyz[:, None, :] + shell[None, :, :]).reshape(-1, 3)
    owner = np.repeat(np.arange(n_at, dtype=np.int32), n_r * n_ang)
    wA = becke_owner_weight(atom_xyz, rp, xyz, owner)
    w = np.tile(wsh, n_at) * wA
    return np.ascontiguousarray(xyz), np.ascontiguousarray(w), owner


def gaussian_potential(pts, n_g, box_lo, box_hi, rng):
    """v(r) = sum_g a_g exp(-|r-c_g|^2/(2 sigma_g^2)), a ~ N(0,1), sigma ~ U(0.5, 2), c ~ U(box)."""
    amp = rng.normal(0.0, 1.0, size=n_g)
    sig = rng.uniform(0.5, 2.0, size=n_g)
    cen = rng.uniform(np.asarray(box_lo, dtype=np.float64), np.asarray(box_hi, dtype=np.float64),
                      size=(n_g, 3))
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.empty(len(pts))
    amp, sig, cen = (np.ascontiguousarray(x) for x in (amp, sig, cen))
    _lib().gg_gaussian_sum(n_g, _dptr(amp), _dptr(cen), _dptr(sig), len(pts), _dptr(pts), _dptr(out))
    return out


def density_matrix(basis, n_occ, d_max, rng):
    """D = C C^T with C ~ N(0,1) of shape [N_b, n_occ]; entries whose centres lie more than
    d_max apart are set to zero (same-atom pairs kept).  Exactly symmetric."""
    ba = basis_atom_index(basis)
    nb = len(ba)
    C = rng.normal(0.0, 1.0, size=(nb, n_occ))
    D = C @ C.T
    D = 0.5 * (D + D.T)
    if d_max is not None:
        xyz = basis["atom_xyz"]
        dd = np.sqrt(((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(axis=2))
        far = dd > d_max
        D[far[ba][:, ba]] = 0.0
    return np.ascontiguousarray(D), C


def energy_weighted_matrix(basis, C, d_max, rng):
    """Q = C diag(e) C^T with seeded level energies e ~ U(-1, -0.05) (occupied levels lie below
    zero), the same coefficients C as D and the same distance cut.  Exactly symmetric."""
    e = np.sort(rng.uniform(-1.0, -0.05, size=C.shape[1]))
    Q = (C * e[None, :]) @ C.T
    Q = 0.5 * (Q + Q.T)
    if d_max is not None:
        ba = basis_atom_index(basis)
        xyz = basis["atom_xyz"]
        dd = np.sqrt(((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(axis=2))
        Q[(dd > d_max)[ba][:, ba]] = 0.0
    return np.ascontiguousarray(Q)


def energy_weighted_for(w, seed: int = 0):
    """Q for a workload that carries its coefficients C (its configuration's distance cut and
    random stream; workloads without a configuration use no cut)."""
    cfg, st = int(w.get("cfg", 0)), int(w.get("structure", 0))
    d_max = CONFIGS[cfg]["d_max"] if cfg in CONFIGS else None
    return energy_weighted_matrix(w["basis"], w["C"], d_max, rng_for(cfg, st, STREAM_ENERGY, seed))


# ----------------------------------------------------------------------------------------------
# configurations

def config_geometry(cfg: int, structure: int = 0) -> np.ndarray:
    rng = rng_for(cfg, structure, STREAM_GEOMETRY)
    if cfg == 1:
        return geometry_random_cube(8, 6.0, 1.0, rng)
    if cfg == 2:
        return geometry_cubic_block(5, 5, 4, 2.2, 0.1, rng)
    if cfg == 3:
        n = int(round(math.exp(rng.uniform(math.log(10.0), math.log(200.0)))))
        return geometry_sc_first_n(n, 2.2, 0.1, rng)
    if cfg == 4:
        return geometry_layered_slab(75, 5, 25.0, rng)
    raise ValueError("unknown configuration %r" % cfg)


def serving_geometry(style: int, n_atoms: int, structure: int) -> np.ndarray:
    """Serving structures: style 2 = jittered simple-cubic block, style 4 = layered slab with the
    window side scaled to 25 sqrt(n/375)."""
    rng = rng_for(5, structure, STREAM_GEOMETRY)
    if style == 2:
        return geometry_sc_first_n(n_atoms, 2.2, 0.1, rng)
    per_layer = max(1, int(round(n_atoms / 5.0)))
    return geometry_layered_slab(per_layer, 5, 25.0 * math.sqrt(n_atoms / 375.0), rng)


def make_workload(atom_xyz, cfg_params, cfg: int, structure: int = 0, iteration: int = 0,
                  with_density=True, n_occ=None, box=None):
    """Build basis, grid, weights, potential and (optionally) D for a geometry."""
    p = cfg_params
    n_at = len(atom_xyz)
    basis = make_basis(atom_xyz, np.zeros(n_at, dtype=np.int32), [p["shells"]], [p["rcut"]], cfg,
                       structure)
    xyz, w, owner = make_grid(atom_xyz, p["rcut"], p["n_r"], p["n_ang"])
    if box is None:
        box = (atom_xyz.min(axis=0), atom_xyz.max(axis=0))
    v = gaussian_potential(xyz, p["n_gauss"], box[0], box[1], rng_for(cfg, structure, STREAM_POTENTIAL))
    out = dict(cfg=cfg, structure=structure, basis=basis, xyz=xyz, w=w, owner=owner, v=v,
               max_batch=p["max_batch"], n_basis=n_basis(basis))
    if with_density:
        occ = n_occ if n_occ is not None else p["n_occ"]
        out["D"], out["C"] = density_matrix(basis, occ, p["d_max"],
                                            rng_for(cfg, structure, STREAM_DENSITY, iteration))
    return out


def config_workload(cfg: int, structure: int = 0, iteration: int = 0, with_density=True):
    """The configuration's synthetic workload (cfg 1-4; cfg 3 takes structure 0..63)."""
    p = CONFIGS[cfg]
    xyz = config_geometry(cfg, structure)
    box = ((0.0, 0.0, 0.0), (6.0, 6.0, 6.0)) if cfg == 1 else None
    n_occ = 2 * len(xyz) if cfg == 3 else None
    return make_workload(xyz, p, cfg, structure, iteration, with_density, n_occ=n_occ, box=box)


# ----------------------------------------------------------------------------------------------
# test inputs

def product_sphere(n_theta: int, n_phi: int):
    """Product angular rule: Gauss-Legendre in cos(theta) x uniform phi (exact for polynomials
    of degree < min(2 n_theta, n_phi) on the sphere)."""
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    ph = (np.arange(n_phi) + 0.5) * (2.0 * math.pi / n_phi)
    z = np.repeat(xg, n_phi)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    p = np.tile(ph, n_theta)
    u = np.stack([s * np.cos(p), s * np.sin(p), z], axis=1)
    w = np.repeat(wg, n_phi) * (2.0 * math.pi / n_phi)
    return u, w


def make_grid_product(atom_xyz, rp, n_r, n_theta, n_phi, r_m: float = R_M):
    """Like make_grid, with the product angular rule instead of the Fibonacci sphere."""
    atom_xyz = np.asarray(atom_xyz, dtype=np.float64)
    r, wr = radial_grid(n_r, r_m)
    u, wa = product_sphere(n_theta, n_phi)
    shell = (r[:, None, None] * u[None, :, :]).reshape(-1, 3)
    wsh = (wr[:, None] * wa[None, :]).reshape(-1)
    n_at = len(atom_xyz)
    xyz = (atom_xyz[:, None, :] + shell[None, :, :]).reshape(-1, 3)
    owner = np.repeat(np.arange(n_at, dtype=np.int32), len(wsh))
    w = np.tile(wsh, n_at) * becke_owner_weight(atom_xyz, rp, xyz, owner)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(w), owner


def gaussian_basis(atom_xyz, shells, alphas, rcut, n_knots=N_KNOTS, rmin=R_MIN):
    """One species per atom; shell j of atom a has radial R(r) = r^l exp(-alpha r^2) (r < rcut,
    unnormalised).  shells[a] / alphas[a] are per-atom lists."""
    shell_ptr, shell_l, shell_radial, rrmin, rrcut, samples = [0], [], [], [], [], []
    for a in range(len(atom_xyz)):
        r = knot_radii(rmin, rcut, n_knots)
        for l, al in zip(shells[a], alphas[a]):
            shell_l.append(int(l))
            shell_radial.append(len(samples))
            rrmin.append(rmin)
            rrcut.append(rcut)
            y = r ** l * np.exp(-al * r * r)
            y[-1] = 0.0
            samples.append(y)
        shell_ptr.append(len(shell_l))
    return dict(
        atom_xyz=np.ascontiguousarray(atom_xyz, dtype=np.float64),
        atom_species=np.arange(len(atom_xyz), dtype=np.int32),
        species_shell_ptr=np.array(shell_ptr, dtype=np.int32),
        shell_l=np.array(shell_l, dtype=np.int32),
        shell_radial=np.array(shell_radial, dtype=np.int32),
        radial_rmin=np.array(rrmin, dtype=np.float64),
        radial_rcut=np.array(rrcut, dtype=np.float64),
        radial_samples=np.ascontiguousarray(np.array(samples, dtype=np.float64)),
        n_knots=int(n_knots),
    )
