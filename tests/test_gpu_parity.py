"""GPU parity: the HIP library through the C ABI against the FP64 oracle.

Bar (FP64 path): batches and lists bit-exact; basis values, H, n and N_e within 1e-12
normwise max relative error (1e-13 for basis values); H exactly symmetric; exact zeros of
n where no basis function reaches.
"""
import sys

import numpy as np
import pytest

from oracle import integrals as oi
from oracle import batching as bt
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


@pytest.fixture(scope="module")
def ctx(nao):
    c = nao.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name", ["config1", "multitile", "two_species"])
def test_batches_and_lists_bit_exact(nao, ctx, name):
    w, B, ref = case(name)
    say("lists", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    perm, bp, lp, li = s.get_batches()
    operm, obp = bt.octree_batches(w["xyz"], w["max_batch"])
    optr, oidx = bt.basis_lists(w["xyz"], operm, obp, B)
    assert np.array_equal(perm, operm) and np.array_equal(bp, obp)
    assert np.array_equal(lp, optr) and np.array_equal(li, oidx)
    s.close()


@pytest.mark.parametrize("name,max_batch", [("two_species", 300), ("two_species", 4096), ("multitile", 1000)])
def test_eval_basis_large_batches(nao, ctx, name, max_batch):
    """Batches of more points than an execution group: each batch is evaluated as one unit whose
    point slices are longer than the basis kernel stages at a time."""
    w, B, ref = case(name)
    say("eval_basis large batches", name, max_batch)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], max_batch)
    perm, bp, lp, li = s.get_batches()
    assert int(np.max(np.diff(bp))) > 256
    phi, ptr = s.eval_basis()
    worst = scale = 0.0
    for b in range(s.n_batches):
        ref_b = oi.batch_phi(B, w["xyz"], perm, bp, lp, li, b)
        got = phi[ptr[b]:ptr[b + 1]].reshape(ref_b.shape)
        if ref_b.size:
            worst = max(worst, float(np.max(np.abs(got - ref_b))))
            scale = max(scale, float(np.max(np.abs(ref_b))))
            assert np.all(got[ref_b == 0.0] == 0.0)
    say("eval_basis large batches", name, max_batch, "abs err", worst, "scale", scale)
    assert worst <= 1e-13 * scale
    s.close()


@pytest.mark.parametrize("name", ["config1", "multitile", "two_species"])
def test_eval_basis_matches_oracle(nao, ctx, name):
    w, B, ref = case(name)
    say("eval_basis", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    perm, bp, lp, li = s.get_batches()
    phi, ptr = s.eval_basis()
    worst = 0.0
    scale = 0.0
    for b in range(s.n_batches):
        ref_b = oi.batch_phi(B, w["xyz"], perm, bp, lp, li, b)
        got = phi[ptr[b]:ptr[b + 1]].reshape(ref_b.shape)
        if ref_b.size:
            worst = max(worst, float(np.max(np.abs(got - ref_b))))
            scale = max(scale, float(np.max(np.abs(ref_b))))
            assert np.all(got[ref_b == 0.0] == 0.0)
    say("eval_basis", name, "abs err", worst, "scale", scale)
    assert worst <= 1e-13 * scale
    s.close()


@pytest.mark.parametrize("name", ["config1", "multitile", "two_species"])
def test_hamiltonian_fp64(nao, ctx, name):
    w, B, ref = case(name)
    say("H fp64", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H = s.integrate_h(w["v"])
    e = rel_max(H, ref["H"])
    say("H fp64", name, "err", e)
    assert e <= TOL
    assert np.array_equal(H, H.T)
    S = s.integrate_h(np.ones(len(w["xyz"])))
    assert rel_max(S, ref["S"]) <= TOL                        # P1: v = 1 gives the overlap
    s.close()


@pytest.mark.parametrize("name", ["config1", "multitile", "two_species"])
def test_density_fp64(nao, ctx, name):
    w, B, ref = case(name)
    say("n fp64", name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    n, Ne = s.update_density(w["D"], electrons=True)
    e = rel_max(n, ref["n"])
    say("n fp64", name, "err", e, "Ne", Ne, ref["Ne"])
    assert e <= TOL
    assert abs(Ne - ref["Ne"]) <= TOL * abs(ref["Ne"])
    assert np.all(n[ref["n"] == 0.0] == 0.0)                  # exact zeros stay exact
    s.close()


def test_identities_on_gpu_outputs(nao, ctx):
    """P3 / P4 on the library's own H, S, n (config 1)."""
    w, B, ref = case("config1")
    say("identities")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H = s.integrate_h(w["v"])
    S = s.integrate_h(np.ones(len(w["xyz"])))
    n, Ne = s.update_density(w["D"], electrons=True)
    D = w["D"]
    assert abs(Ne - float(np.sum(D * S))) <= 1e-12 * abs(Ne)
    lhs, rhs = float(np.sum(D * H)), float(np.dot(w["w"] * w["v"], n))
    assert abs(lhs - rhs) <= 1e-12 * float(np.sum(np.abs(D * H)))
    s.close()


@pytest.mark.parametrize("group_max", [0, 16, 48, 128, 256])
def test_grouping_invariance(nao, ctx, group_max):
    """P7 on the GPU: execution grouping changes only summation order."""
    w, B, ref = case("multitile")
    say("grouping", group_max)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    s.set_group_max(group_max)
    assert rel_max(s.integrate_h(w["v"]), ref["H"]) <= TOL
    assert rel_max(s.update_density(w["D"]), ref["n"]) <= TOL
    s.close()


@pytest.mark.parametrize("max_batch", [1, 7, 64, 4096])
def test_batch_size_edge_cases(nao, ctx, max_batch):
    """Batches of one point, ragged sizes and a batch larger than an execution group."""
    w, B, ref = case("two_species")
    say("max_batch", max_batch)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], max_batch)
    assert rel_max(s.integrate_h(w["v"]), ref["H"]) <= TOL
    assert rel_max(s.update_density(w["D"]), ref["n"]) <= TOL
    s.close()


def test_density_reads_upper_triangle(nao, ctx):
    w, B, ref = case("multitile")
    say("upper triangle")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    D = w["D"].copy()
    D[np.tril_indices(len(D), -1)] = 12345.0
    assert rel_max(s.update_density(D), ref["n"]) <= TOL
    s.close()


def test_nonsymmetric_density_matrix_reads_upper_triangle(nao, ctx):
    """For a D that is not symmetric the result is that of the symmetric matrix whose upper
    triangle is D's (the lower triangle is never read), for the density and its gradient."""
    w, B, ref = case("two_species")
    say("non-symmetric D")
    rng = np.random.default_rng(77)
    D = rng.normal(size=w["D"].shape)
    Du = oi.symmetric_from_upper(D)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    n_ref = oi.density(B, w["xyz"], Du)
    assert rel_max(s.update_density(D), n_ref) <= TOL
    n, gn = s.update_density_gradient(D)
    n2, g_ref = oi.density_gradient(B, w["xyz"], Du)
    assert rel_max(n, n_ref) <= TOL and rel_max(gn, g_ref) <= TOL
    # not (D + D^T) / 2: that reading gives a different density here
    assert rel_max(oi.density(B, w["xyz"], 0.5 * (D + D.T)), n_ref) > 1e-3
    s.close()


def test_device_memspace_matches_host(nao, ctx):
    import torch
    w, B, ref = case("multitile")
    say("device memspace")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    v = torch.from_numpy(w["v"]).cuda()
    D = torch.from_numpy(w["D"]).cuda()
    H = torch.empty((s.n_basis, s.n_basis), dtype=torch.float64, device="cuda")
    n = torch.empty(s.n_points, dtype=torch.float64, device="cuda")
    s.integrate_h(v, out=H)
    s.update_density(D, out=n)
    ctx.synchronize()
    assert rel_max(H.cpu().numpy(), ref["H"]) <= TOL
    assert rel_max(n.cpu().numpy(), ref["n"]) <= TOL
    phi_dev = torch.empty(int(s.eval_basis()[1][-1]), dtype=torch.float64, device="cuda")
    phi_host, ptr = s.eval_basis()
    s.eval_basis(out=phi_dev)
    ctx.synchronize()
    assert np.array_equal(phi_dev.cpu().numpy(), phi_host)
    s.close()


def test_empty_system(nao, ctx):
    w, B, ref = case("config1")
    say("empty")
    s = nao.build_batches(ctx, w["basis"], np.zeros((0, 3)), np.zeros(0), 200)
    H = s.integrate_h(np.zeros(0))
    assert H.shape == (40, 40) and np.all(H == 0.0)
    n, Ne = s.update_density(w["D"], electrons=True)
    assert n.shape == (0,) and Ne == 0.0
    s.close()


def test_invalid_arguments_return_codes(nao, ctx):
    w, B, ref = case("config1")
    say("invalid args")
    with pytest.raises(nao.NaoError) as e:
        nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], 0)
    assert e.value.status == nao.ERR_INVALID_ARG
    bad = dict(w["basis"])
    bad["shell_l"] = np.array([0, 0, 4], np.int32)
    with pytest.raises(nao.NaoError):
        nao.build_batches(ctx, bad, w["xyz"], w["w"], 200)
    wneg = w["w"].copy()
    wneg[3] = -1.0
    with pytest.raises(nao.NaoError):
        nao.build_batches(ctx, w["basis"], w["xyz"], wneg, 200)
    # the context stays usable after argument errors
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], 200)
    assert rel_max(s.integrate_h(w["v"]), ref["H"]) <= TOL
    s.close()


@pytest.mark.parametrize("overlap", ["1", "0"])
def test_small_blocks(nao, monkeypatch, overlap):
    """Basis values in blocks of at most 16 MB, several per operation: the basis evaluation of
    block k + 1 overlapped with the contraction of block k on a second stream (NAO_OVERLAP=1, the
    default) or the two serial on one stream (0); both against the oracle."""
    w, B, ref = case("multitile")
    monkeypatch.setenv("NAO_SCRATCH_MB", "16")
    monkeypatch.setenv("NAO_OVERLAP", overlap)
    say("small blocks, overlap", overlap)
    c = nao.Context(0)
    c.profile(True)
    s = nao.build_batches(c, w["basis"], w["xyz"], w["w"], w["max_batch"])
    for prec, tol in (("fp64", TOL), ("fp32", 1e-6)):
        for rep in range(2):  # the second call reuses the buffers and the events
            eH = rel_max(s.integrate_h(w["v"], precision=prec), ref["H"])
            en = rel_max(s.update_density(w["D"], precision=prec), ref["n"])
            say("small blocks, overlap", overlap, prec, rep, "H %.2e n %.2e" % (eH, en))
            assert eH <= tol and en <= tol
    prof = c.profile_read()
    say("small blocks, overlap", overlap, "launches", prof)
    assert prof["basis_f64"][0] >= 4 * 3  # four operations of three or more blocks each
    s.close()
    c.close()


def test_small_blocks_budget_without_room_for_overlap(nao, monkeypatch):
    """A budget that holds the system and one basis buffer but not the second: the calls run
    their blocks serially (no error) and still equal the oracle."""
    import ctypes
    w, B, ref = case("multitile")
    monkeypatch.setenv("NAO_SCRATCH_MB", "16")
    monkeypatch.setenv("NAO_OVERLAP", "0")
    probe = nao.Context(0)
    s = nao.build_batches(probe, w["basis"], w["xyz"], w["w"], w["max_batch"])
    s.integrate_h(w["v"])
    s.update_density(w["D"])
    used, budget = ctypes.c_size_t(), ctypes.c_size_t()
    assert nao._lib.nao_ctx_memory(probe.handle, ctypes.byref(used), ctypes.byref(budget)) == 0
    s.close()
    probe.close()
    monkeypatch.setenv("NAO_OVERLAP", "1")
    say("small blocks, budget without room for the second buffer")
    c = nao.Context(0, hbm_budget=int(used.value) + (1 << 20))
    c.profile(True)
    s = nao.build_batches(c, w["basis"], w["xyz"], w["w"], w["max_batch"])
    for rep in range(2):
        assert rel_max(s.integrate_h(w["v"]), ref["H"]) <= TOL
        assert rel_max(s.update_density(w["D"]), ref["n"]) <= TOL
    assert c.profile_read()["basis_f64"][0] >= 4 * 3  # four calls of three or more blocks
    used2 = ctypes.c_size_t()
    assert nao._lib.nao_ctx_memory(c.handle, ctypes.byref(used2), ctypes.byref(budget)) == 0
    assert used2.value <= budget.value
    s.close()
    c.close()


def test_small_blocks_extended_operations(nao, monkeypatch):
    """The density gradient, the Hamiltonian with a field and with the kinetic term, and the local
    Pulay forces over blocks of at most 16 MB of basis values: with the overlap (basis values and
    their extra values in two buffers, basis launches on a second stream) equal to the serial
    loop up to the order of the FP64 atomics, on two calls in a row, in FP64 and FP32."""
    from workloads.generate import energy_weighted_for
    w, B, ref = case("multitile")
    monkeypatch.setenv("NAO_SCRATCH_MB", "16")
    a = 0.3 * np.random.default_rng(31).normal(size=(len(w["xyz"]), 3))
    Q = energy_weighted_for(w, 1)
    out = {}
    for overlap in ("1", "0"):
        monkeypatch.setenv("NAO_OVERLAP", overlap)
        c = nao.Context(0)
        c.profile(True)
        s = nao.build_batches(c, w["basis"], w["xyz"], w["w"], w["max_batch"])
        for prec in ("fp64", "fp32"):
            for rep in range(2):
                say("small blocks, extended operations, overlap", overlap, prec, rep)
                n, gn = s.update_density_gradient(w["D"], precision=prec)
                r = (n, gn, s.integrate_h_gga(w["v"], a, precision=prec),
                     s.integrate_h_ks(w["v"], precision=prec), s.pulay_forces(w["D"], Q, w["v"], precision=prec))
                if rep == 0:
                    out[(overlap, prec)] = r
                else:  # the second call reuses the buffers and events
                    for x, y in zip(r, out[(overlap, prec)]):
                        assert rel_max(x, y) <= 1e-13
        prof = c.profile_read()
        assert prof["basis_grad_f64"][0] >= 2 * 3  # three or more blocks per call
        s.close()
        c.close()
    for prec in ("fp64", "fp32"):
        tol = 1e-12  # FP32 tile sums are the same; only the order of the FP64 atomics differs
        names = ("n", "grad n", "H with a field", "H with the kinetic term", "forces")
        for nm, x, y in zip(names, out[("1", prec)], out[("0", prec)]):
            e = rel_max(x, y)
            say("small blocks, extended operations", prec, nm, "overlap vs serial %.2e" % e)
            assert e <= tol


# Stated error bounds of the reduced-precision modes against the FP64 oracle (normwise max
# relative error of H, n and N_e); the measured values are printed for the record.
PREC_TOL = {"fp32": 1e-6, "bf16x3": 3e-5, "bf16x6": 1e-6}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", ["config1", "multitile"])
def test_reduced_precision_error(nao, ctx, name, prec):
    w, B, ref = case(name)
    say("precision", prec, name)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H = s.integrate_h(w["v"], precision=prec)
    n, Ne = s.update_density(w["D"], precision=prec, electrons=True)
    eH, en = rel_max(H, ref["H"]), rel_max(n, ref["n"])
    eN = abs(Ne - ref["Ne"]) / abs(ref["Ne"])
    say("precision", prec, name, "e_H %.3e e_n %.3e e_Ne %.3e" % (eH, en, eN))
    assert np.array_equal(H, H.T)
    assert np.all(n[ref["n"] == 0.0] == 0.0)
    tol = PREC_TOL[prec]
    assert eH <= tol and en <= tol and eN <= tol
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["config1", "multitile"])
def test_wide_hamiltonian_tiles(nao, ctx, name, prec):
    """128-wide Hamiltonian tiles give the same H (FP64: within 1e-12 of the oracle; other
    modes: equal to the 64-wide result within their own error)."""
    w, B, ref = case(name)
    say("h_tile 128", name, prec)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    H64 = s.integrate_h(w["v"], precision=prec)
    n64 = s.update_density(w["D"], precision=prec)
    s.set_h_tile(128)
    H128 = s.integrate_h(w["v"], precision=prec)
    n128 = s.update_density(w["D"], precision=prec)
    assert np.array_equal(H128, H128.T)
    if prec == "fp64":
        assert rel_max(H128, ref["H"]) <= TOL and rel_max(n128, ref["n"]) <= TOL
    else:
        assert rel_max(H128, H64) <= 1e-5 and rel_max(n128, n64) <= 1e-12
    s.close()


def test_autotune_choice_and_cache(nao, ctx, tmp_path, monkeypatch):
    """The autotuner keeps results exact, writes its cache, and a second system of the same
    shape class takes the cached choice without timing."""
    w, B, ref = case("multitile")
    say("autotune")
    monkeypatch.setenv("NAO_TUNE_CACHE", str(tmp_path / "tune.json"))
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    ht, gm, ms = s.autotune(w["v"], w["D"], precision="fp64", force=True)
    assert ht in (64, 128) and gm in (128, 192, 256) and ms > 0
    assert rel_max(s.integrate_h(w["v"]), ref["H"]) <= TOL
    assert rel_max(s.update_density(w["D"]), ref["n"]) <= TOL
    text = (tmp_path / "tune.json").read_text()
    assert "fp64" in text and str(ht) in text
    s2 = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    ht2, gm2, ms2 = s2.autotune(w["v"], w["D"], precision="fp64")
    assert (ht2, gm2, ms2) == (ht, gm, -1.0)
    s.close()
    s2.close()
