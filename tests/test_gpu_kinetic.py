"""Kohn-Sham Hamiltonian with the kinetic term on the GPU against the oracle: element by element
on the small cases (several tiles, ragged tails, two species with l = 3), with and without a
vector field, the kinetic matrix alone, grouping invariance, FP32 error, memory spaces and
argument errors."""
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


def field(name, n):
    seed = {"config1": 1, "multitile": 2, "two_species": 3}[name]
    return 0.3 * np.random.default_rng(700 + seed).normal(size=(n, 3))


@functools.lru_cache(maxsize=None)
def ref_ks(name, with_field):
    w, B, ref = case(name)
    a = field(name, len(w["xyz"])) if with_field else None
    return oi.hamiltonian_ks(B, w["xyz"], w["w"], w["v"], a)


@functools.lru_cache(maxsize=None)
def ref_kinetic(name):
    w, B, ref = case(name)
    return oi.kinetic(B, w["xyz"], w["w"])


@pytest.mark.parametrize("name", CASES)
def test_ks_hamiltonian_fp64_matches_oracle(nao, ctx, name):
    w, B, ref = case(name)
    say("kohn-sham hamiltonian fp64", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H0 = s.integrate_h_ks(w["v"])
    H1 = s.integrate_h_ks(w["v"], field(name, len(w["xyz"])))
    T = s.integrate_h_ks(np.zeros_like(w["v"]))
    e0, e1 = rel_max(H0, ref_ks(name, False)), rel_max(H1, ref_ks(name, True))
    eT = rel_max(T, ref_kinetic(name))
    say("kohn-sham hamiltonian fp64", name, "e_H %.3e, with field %.3e, kinetic alone %.3e" % (e0, e1, eT))
    assert e0 <= 1e-12 and e1 <= 1e-12 and eT <= 1e-12
    assert np.array_equal(H0, H0.T) and np.array_equal(H1, H1.T)
    s.close()


def test_ks_hamiltonian_grouping_and_fp32(nao, ctx):
    w, B, ref = case("multitile")
    a = field("multitile", len(w["xyz"]))
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H0 = s.integrate_h_ks(w["v"], a)
    for gm in (0, 48):
        s.set_group_max(gm)
        assert rel_max(s.integrate_h_ks(w["v"], a), H0) <= 1e-13
    s.set_group_max(256)
    e32 = rel_max(s.integrate_h_ks(w["v"], a, precision="fp32"), ref_ks("multitile", True))
    say("kohn-sham hamiltonian fp32 multitile e_H %.3e" % e32)
    assert e32 <= 1e-5
    with pytest.raises(nao.NaoError):
        s.integrate_h_ks(w["v"], a, precision="bf16x3")
    s.close()


def test_ks_hamiltonian_device_memspace(nao, ctx):
    import torch
    w, B, ref = case("config1")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    dev = torch.device("cuda:0")
    v = torch.from_numpy(w["v"]).to(dev)
    H = torch.empty((s.n_basis, s.n_basis), dtype=torch.float64, device=dev)
    s.integrate_h_ks(v, out=H)
    ctx.synchronize()
    assert rel_max(H.cpu().numpy(), ref_ks("config1", False)) <= 1e-12
    with pytest.raises(ValueError):
        s.integrate_h_ks(v, field("config1", len(w["xyz"])))
    s.close()
