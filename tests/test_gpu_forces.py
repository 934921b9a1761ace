"""Local Pulay forces on the GPU against the oracle: F element by element on the small cases
(several tiles, ragged tails, two species with l = 3), the sum over atoms against the GPU
density gradients of D and Q, grouping invariance, the vanishing case, FP32 error, memory
spaces and argument errors."""
import functools
import sys

import numpy as np
import pytest

from oracle import integrals as oi
from tests.gpu_cases import case, rel_max
from workloads import generate as g

pytestmark = pytest.mark.gpu

CASES = ["config1", "multitile", "two_species"]

# stated FP32 accuracy of the forces (normwise max relative): the two products accumulate in
# FP32 over the whole list before the FP64 column sums
FP32_TOL = 1e-5


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


@functools.lru_cache(maxsize=None)
def q_of(name):
    w, B, ref = case(name)
    return g.energy_weighted_for(w, 1)


@functools.lru_cache(maxsize=None)
def ref_forces(name):
    w, B, ref = case(name)
    return oi.pulay_forces(B, w["xyz"], w["w"], w["v"], w["D"], q_of(name))


@pytest.mark.parametrize("name", CASES)
def test_forces_fp64_matches_oracle(nao, ctx, name):
    w, B, ref = case(name)
    say("forces fp64", name)
    Q = q_of(name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    F = s.pulay_forces(w["D"], Q, w["v"])
    e = rel_max(F, ref_forces(name))
    say("forces fp64", name, "e_F %.3e, max|F| %.3e" % (e, float(np.max(np.abs(F)))))
    assert F.shape == (len(B.atom_xyz), 3)
    assert e <= 1e-12
    # sum over atoms: the local-potential and q parts equal sum_p w_p [v_p grad n_D - grad n_Q]
    # from the GPU's own gradients; the kinetic part is the oracle's
    _, gD = s.update_density_gradient(w["D"])
    _, gQ = s.update_density_gradient(Q)
    tot = ((w["w"] * w["v"])[:, None] * gD - w["w"][:, None] * gQ).sum(axis=0)
    kin = (ref_forces(name) - oi.pulay_forces(B, w["xyz"], w["w"], w["v"], w["D"], Q, kinetic=False)).sum(axis=0)
    assert float(np.max(np.abs(F.sum(axis=0) - tot - kin))) <= 1e-12 * float(np.max(np.abs(F)))
    s.close()


def test_forces_grouping_invariance_and_zero_case(nao, ctx):
    w, B, ref = case("multitile")
    Q = q_of("multitile")
    say("forces grouping")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    F0 = s.pulay_forces(w["D"], Q, w["v"])
    for gm in (0, 48):
        s.set_group_max(gm)
        assert rel_max(s.pulay_forces(w["D"], Q, w["v"]), F0) <= 1e-13
    s.set_group_max(256)
    # no density matrices: no force, whatever the potential
    assert np.all(s.pulay_forces(np.zeros_like(Q), np.zeros_like(Q), w["v"]) == 0.0)
    s.close()


@pytest.mark.parametrize("name", ["config1", "multitile"])
def test_forces_fp32_error(nao, ctx, name):
    w, B, ref = case(name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    F = s.pulay_forces(w["D"], q_of(name), w["v"], precision="fp32")
    e = rel_max(F, ref_forces(name))
    say("forces fp32", name, "e_F %.3e" % e)
    assert e <= FP32_TOL
    s.close()


def test_forces_device_memspace_and_errors(nao, ctx):
    import torch
    w, B, ref = case("config1")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    dev = torch.device("cuda:0")
    D = torch.from_numpy(w["D"]).to(dev)
    Q = torch.from_numpy(q_of("config1")).to(dev)
    v = torch.from_numpy(w["v"]).to(dev)
    F = torch.empty((len(B.atom_xyz), 3), dtype=torch.float64, device=dev)
    s.pulay_forces(D, Q, v, out=F)
    ctx.synchronize()
    assert rel_max(F.cpu().numpy(), ref_forces("config1")) <= 1e-12
    with pytest.raises(nao.NaoError):
        s.pulay_forces(w["D"], q_of("config1"), w["v"], precision="bf16x6")
    with pytest.raises(ValueError):
        s.pulay_forces(D, q_of("config1"), w["v"])
    s.close()
