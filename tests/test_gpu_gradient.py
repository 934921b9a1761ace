"""Density gradient on the GPU against the oracle: grad n = 2 grad(Phi)^T D Phi element by
element on the small cases (several tiles, ragged tails, two species with l = 3), the density
of the same call against nao_update_density, grouping invariance, FP32 error, memory spaces
and argument errors."""
import functools
import sys

import numpy as np
import pytest

from oracle import integrals as oi
from tests.gpu_cases import case, rel_max

pytestmark = pytest.mark.gpu

CASES = ["config1", "multitile", "two_species"]


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
def ref_gradient(name):
    w, B, ref = case(name)
    return oi.density_gradient(B, w["xyz"], w["D"])


@pytest.mark.parametrize("name", CASES)
def test_gradient_fp64_matches_oracle(nao, ctx, name):
    w, B, ref = case(name)
    say("gradient fp64", name)
    n_ref, g_ref = ref_gradient(name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    n, g = s.update_density_gradient(w["D"])
    en, eg = rel_max(n, n_ref), rel_max(g, g_ref)
    say("gradient fp64", name, "e_n %.3e e_grad %.3e" % (en, eg))
    assert en <= 1e-12 and eg <= 1e-12
    assert np.all(g[n_ref == 0.0] == 0.0)
    assert rel_max(n, s.update_density(w["D"])) <= 1e-12
    s.close()


def test_gradient_grouping_invariance(nao, ctx):
    w, B, ref = case("multitile")
    say("gradient grouping")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    n0, g0 = s.update_density_gradient(w["D"])
    for gm in (0, 48):
        s.set_group_max(gm)
        n1, g1 = s.update_density_gradient(w["D"])
        assert rel_max(n1, n0) <= 1e-13 and rel_max(g1, g0) <= 1e-13
    s.close()


@pytest.mark.parametrize("name", ["config1", "multitile"])
def test_gradient_fp32_error(nao, ctx, name):
    w, B, ref = case(name)
    n_ref, g_ref = ref_gradient(name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    n, g = s.update_density_gradient(w["D"], precision="fp32")
    en, eg = rel_max(n, n_ref), rel_max(g, g_ref)
    say("gradient fp32", name, "e_n %.3e e_grad %.3e" % (en, eg))
    assert en <= 1e-5 and eg <= 1e-5
    s.close()


def test_gradient_device_memspace_and_errors(nao, ctx):
    import torch
    w, B, ref = case("config1")
    n_ref, g_ref = ref_gradient("config1")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    dev = torch.device("cuda:0")
    D = torch.from_numpy(w["D"]).to(dev)
    n = torch.empty(s.n_points, dtype=torch.float64, device=dev)
    g = torch.empty((s.n_points, 3), dtype=torch.float64, device=dev)
    s.update_density_gradient(D, out=n, out_grad=g)
    ctx.synchronize()
    assert rel_max(g.cpu().numpy(), g_ref) <= 1e-12 and rel_max(n.cpu().numpy(), n_ref) <= 1e-12
    with pytest.raises(nao.NaoError):
        s.update_density_gradient(w["D"], precision="bf16x3")
    s.close()


def field(name, n):
    """Seeded vector field a [n, 3] (input of the Hamiltonian with a vector field)."""
    seed = {"config1": 1, "multitile": 2, "two_species": 3}[name]
    return 0.3 * np.random.default_rng(500 + seed).normal(size=(n, 3))


@functools.lru_cache(maxsize=None)
def ref_gga(name):
    w, B, ref = case(name)
    return oi.hamiltonian_gga(B, w["xyz"], w["w"], w["v"], field(name, len(w["xyz"])))


@pytest.mark.parametrize("name", CASES)
def test_gga_hamiltonian_fp64_matches_oracle(nao, ctx, name):
    w, B, ref = case(name)
    say("gga hamiltonian fp64", name)
    a = field(name, len(w["xyz"]))
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H = s.integrate_h_gga(w["v"], a)
    e = rel_max(H, ref_gga(name))
    say("gga hamiltonian fp64", name, "e_H %.3e" % e)
    assert e <= 1e-12
    assert np.array_equal(H, H.T)
    # without the field it is the local Hamiltonian
    assert rel_max(s.integrate_h_gga(w["v"], np.zeros_like(a)), ref["H"]) <= 1e-12
    s.close()


def test_gga_hamiltonian_grouping_and_fp32(nao, ctx):
    w, B, ref = case("multitile")
    a = field("multitile", len(w["xyz"]))
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H0 = s.integrate_h_gga(w["v"], a)
    s.set_group_max(0)
    assert rel_max(s.integrate_h_gga(w["v"], a), H0) <= 1e-13
    s.set_group_max(256)
    e32 = rel_max(s.integrate_h_gga(w["v"], a, precision="fp32"), ref_gga("multitile"))
    say("gga hamiltonian fp32 multitile e_H %.3e" % e32)
    assert e32 <= 1e-5
    with pytest.raises(nao.NaoError):
        s.integrate_h_gga(w["v"], a, precision="bf16x6")
    s.close()
