"""The basis kernel's off-chip branches against the oracle: a spline table larger than the kernel
stages in LDS and more shells than it stages (nine species of 15 shells: 135 radial functions),
units with more atoms than it stages (a 343-atom dense cluster); beside them the two-species basis
with 8 radial functions each of a two-element slab, whose table is staged on chip.  Every
operation that evaluates basis values is checked: basis values, H and n in FP64 and FP32, the
density gradient, the Kohn-Sham Hamiltonian with a field, and the many-structure launch."""
import functools
import sys

import numpy as np
import pytest

from oracle import integrals as oi
from tests.gpu_cases import case, rel_max

pytestmark = pytest.mark.gpu

CASES = ["two_species_8", "dense_cluster", "many_species"]
SPLINE_LDS_DOUBLES = 8192   # table size the basis kernel stages in LDS
STAGED_ATOMS, STAGED_SHELLS = 192, 128


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
    return 0.3 * np.random.default_rng(900 + CASES.index(name)).normal(size=(n, 3))


@functools.lru_cache(maxsize=None)
def refs(name):
    w, B, ref = case(name)
    n, gn = oi.density_gradient(B, w["xyz"], w["D"])
    ks = oi.hamiltonian_ks(B, w["xyz"], w["w"], w["v"], field(name, len(w["xyz"])))
    return n, gn, ks


@pytest.mark.parametrize("name", CASES)
def test_basis_values_and_contractions(nao, ctx, name):
    w, B, ref = case(name)
    say("off-chip basis", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    perm, bp, lp, li = s.get_batches()
    phi, ptr = s.eval_basis()
    worst = scale = 0.0
    for b in range(0, s.n_batches, max(1, s.n_batches // 40)):
        rb = oi.batch_phi(B, w["xyz"], perm, bp, lp, li, b)
        got = phi[ptr[b]:ptr[b + 1]].reshape(rb.shape)
        if rb.size:
            worst = max(worst, float(np.max(np.abs(got - rb))))
            scale = max(scale, float(np.max(np.abs(rb))))
    eH, en = rel_max(s.integrate_h(w["v"]), ref["H"]), rel_max(s.update_density(w["D"]), ref["n"])
    eH32 = rel_max(s.integrate_h(w["v"], precision="fp32"), ref["H"])
    en32 = rel_max(s.update_density(w["D"], precision="fp32"), ref["n"])
    say("off-chip basis", name, "phi %.2e (scale %.2e), H %.2e, n %.2e, fp32 H %.2e n %.2e" % (
        worst, scale, eH, en, eH32, en32))
    assert worst <= 1e-13 * scale
    assert eH <= 1e-12 and en <= 1e-12
    assert eH32 <= 1e-5 and en32 <= 1e-5
    s.close()


@pytest.mark.parametrize("name", CASES)
def test_gradient_and_ks_hamiltonian(nao, ctx, name):
    w, B, ref = case(name)
    n_ref, g_ref, ks_ref = refs(name)
    say("off-chip gradient / kohn-sham", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    n, gn = s.update_density_gradient(w["D"])
    Hks = s.integrate_h_ks(w["v"], field(name, len(w["xyz"])))
    en, eg, eks = rel_max(n, n_ref), rel_max(gn, g_ref), rel_max(Hks, ks_ref)
    say("off-chip gradient / kohn-sham", name, "n %.2e grad n %.2e H_KS %.2e" % (en, eg, eks))
    assert en <= 1e-12 and eg <= 1e-12 and eks <= 1e-12
    s.close()


def test_many_structure_launch(nao, ctx):
    """nao_run_many over the three cases at once (no spline staging: one table does not fit)."""
    import torch
    dev = torch.device("cuda:0")
    systems, outs, work = [], [], []
    for name in CASES:
        w, B, ref = case(name)
        s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
        v = torch.from_numpy(w["v"]).to(dev)
        D = torch.from_numpy(w["D"]).to(dev)
        H = torch.empty((s.n_basis, s.n_basis), dtype=torch.float64, device=dev)
        n = torch.empty(s.n_points, dtype=torch.float64, device=dev)
        systems.append(s)
        outs.append((v, D, H, n, ref))
        work += [(s, "h", v, H), (s, "n", D, n)]
    torch.cuda.synchronize()
    say("off-chip many-structure launch")
    ctx.run_many(work)
    ctx.synchronize()
    for name, (v, D, H, n, ref) in zip(CASES, outs):
        eH, en = rel_max(H.cpu().numpy(), ref["H"]), rel_max(n.cpu().numpy(), ref["n"])
        say("off-chip many-structure launch", name, "H %.2e n %.2e" % (eH, en))
        assert eH <= 1e-12 and en <= 1e-12
    for s in systems:
        s.close()
