"""Edge cases of the extended operations (density gradient, Hamiltonian with a field or the
kinetic term, local Pulay forces): a structure without points, and an atom whose functions
reach no point (its forces, matrix rows and gradient contributions are exact zeros), against
the oracle."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import integrals as oi
from tests.gpu_cases import case, rel_max
from workloads import generate as g

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nao():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_06636_amd import nao as lib
    return lib


@pytest.fixture(scope="module")
def ctx(nao):
    c = nao.Context(0)
    yield c
    c.close()


def test_extended_operations_without_points(nao, ctx):
    w, B, ref = case("config1")
    say("extended operations, empty system")
    s = nao.build_batches(ctx, w["basis"], np.zeros((0, 3)), np.zeros(0), 200)
    nb, na = w["D"].shape[0], len(B.atom_xyz)
    n, gn = s.update_density_gradient(w["D"])
    assert n.shape == (0,) and gn.shape == (0, 3)
    for H in (s.integrate_h_gga(np.zeros(0), np.zeros((0, 3))), s.integrate_h_ks(np.zeros(0)),
              s.integrate_h_ks(np.zeros(0), np.zeros((0, 3)))):
        assert H.shape == (nb, nb) and np.all(H == 0.0)
    F = s.pulay_forces(w["D"], w["D"], np.zeros(0))
    assert F.shape == (na, 3) and np.all(F == 0.0)
    s.close()


def far_atom_case():
    """config-1 structure plus one atom 60 A away from every grid point."""
    w, B, ref = case("config1")
    xyz = np.concatenate([w["basis"]["atom_xyz"], [[60.0, 60.0, 60.0]]])
    species = np.concatenate([w["basis"]["atom_species"], [0]]).astype(np.int32)
    basis = dict(w["basis"], atom_xyz=xyz, atom_species=species)
    nb = g.n_basis(basis)
    rng = np.random.default_rng(31)
    C = rng.normal(size=(nb, 6))
    D = C @ C.T
    Q = (C * rng.uniform(-1.0, -0.1, 6)) @ C.T
    return basis, w, D, 0.5 * (Q + Q.T)


def test_atom_without_points(nao, ctx):
    basis, w, D, Q = far_atom_case()
    B = ob.Basis(basis)
    say("extended operations, atom without points")
    far = np.arange(B.atom_first[-2], B.atom_first[-1])
    s = nao.build_batches(ctx, basis, w["xyz"], w["w"], w["max_batch"])
    F = s.pulay_forces(D, Q, w["v"])
    Fref = oi.pulay_forces(B, w["xyz"], w["w"], w["v"], D, Q)
    assert rel_max(F, Fref) <= 1e-12 and np.all(F[-1] == 0.0)
    H = s.integrate_h_ks(w["v"])
    Href = oi.hamiltonian_ks(B, w["xyz"], w["w"], w["v"])
    assert rel_max(H, Href) <= 1e-12
    assert np.all(H[far] == 0.0) and np.all(H[:, far] == 0.0)
    n, gn = s.update_density_gradient(D)
    nref, gref = oi.density_gradient(B, w["xyz"], D)
    assert rel_max(n, nref) <= 1e-12 and rel_max(gn, gref) <= 1e-12
    say("atom without points: e_F %.3e e_H %.3e e_grad %.3e" % (rel_max(F, Fref), rel_max(H, Href), rel_max(gn, gref)))
    s.close()
