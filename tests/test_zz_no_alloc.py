"""Allocation-free Hamiltonian integration (nao_integrate_h_noalloc) against nao_integrate_h.

Both calls go through the C ABI on the same seeded inputs.  Two systems are integrated in a
row, the second smaller than the first, so the second call runs over what the first left in
the fixed scratch.  Bar: the two entry points agree to 1e-12 (normwise max relative error)
in every precision, and the FP64 result is within 1e-12 of the oracle.
"""
import sys

import numpy as np
import pytest

from tests.gpu_cases import case, rel_max

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nao():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_06636_amd import nao as lib
    return lib


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x6"])
def test_noalloc_matches_integrate_h(nao, precision):
    import torch
    ctx = nao.Context(0)
    try:
        for name in ("multitile", "config1"):  # the second call is the smaller input
            w, B, ref = case(name)
            say("integrate_h_noalloc", name, precision)
            s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
            v = torch.from_numpy(w["v"]).to("cuda:0")
            nb = s.n_basis
            H_ref = torch.full((nb, nb), np.nan, dtype=torch.float64, device="cuda:0")
            H_na = torch.full((nb, nb), np.nan, dtype=torch.float64, device="cuda:0")
            s.integrate_h(v, precision=precision, out=H_ref)
            s.integrate_h_noalloc(v, H_na, precision=precision)
            ctx.synchronize()
            a, b = H_na.cpu().numpy(), H_ref.cpu().numpy()
            assert np.isfinite(a).all()
            assert np.array_equal(a, a.T)
            e = rel_max(a, b)
            say("  vs nao_integrate_h %.2e" % e)
            assert e <= TOL
            if precision == "fp64":
                eo = rel_max(a, ref["H"])
                say("  vs oracle %.2e" % eo)
                assert eo <= TOL
            s.close()
    finally:
        ctx.close()


def test_noalloc_rejects_host_memory(nao):
    import torch
    ctx = nao.Context(0)
    try:
        w, B, ref = case("config1")
        s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
        H = torch.empty((s.n_basis, s.n_basis), dtype=torch.float64, device="cuda:0")
        with pytest.raises(ValueError):
            s.integrate_h_noalloc(w["v"], H)
        s.close()
    finally:
        ctx.close()
