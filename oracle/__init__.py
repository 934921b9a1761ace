"""Plain FP64 CPU oracle for the real-space grid operations -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  The HIP library never imports, links or calls it, and it never
imports the library: the two share no code.  The only shared module is the
seeded input generator in workloads/, which holds none of the method's
arithmetic.

What it computes (Huhn et al., "GPGPU Acceleration of All-Electron Electronic
Structure Theory Using Localized Numeric Atom-Centered Basis Functions"):

* spline.py    -- numeric radial functions as natural cubic splines on a
                  logarithmic grid (the NAO radial parts of Section
                  "Computational Choices in FHI-aims").
* ylm.py       -- real orthonormal spherical harmonics, l <= 3.
* basis.py     -- phi_i(r) = R_s(|r - R_A|) Y_lm(unit(r - R_A)), the basis
                  functions of eq. (EVNonPeriodic).
* batching.py  -- octree batches of grid points (Section "Grid Partitioning")
                  and the per-batch relevant-basis lists nnz(B_nu) (Section
                  "Parallelization and Dimensionality Reduction").
* integrals.py -- the quadrature h_ij = sum_r w(r) phi_i(r) v(r) phi_j(r)
                  (eq. H_int_aims with a local potential), the density
                  n(r) = sum_ij phi_i(r) n_ij phi_j(r) (eq. Density), the
                  electron count and the overlap s_ij (eq. OverlapNoPeriodic).

Readings taken where the paper is silent (spline variable and boundary
conditions, harmonic convention, octree tie rules, relevance test) are stated
in each module's docstring.

Parity status: every function here is pinned by tests in
tests/test_oracle_*.py against closed forms, library routines (scipy),
identities or brute force.  Nothing here is "parity unpinned".
"""
from . import batching, basis, integrals, spline, ylm  # noqa: F401
