"""Many structures in one launch sequence (nao_run_many): each result equals the structure's
own single-call result within FP64 summation-order tolerance, graph replays equal the eager
launch on every replay, and the mixed list matches the oracle for one member."""
import sys

import numpy as np
import pytest

from tests.gpu_cases import case, rel_max
from workloads import generate as g

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_06636_amd import nao
    ctx = nao.Context(0)
    structs = []
    for k in range(5):   # config-3-like structures on a reduced 12 x 38 grid
        xyz = g.geometry_sc_first_n([6, 11, 19, 27, 8][k], 2.2, 0.1, g.rng_for(3, 200 + k, 0))
        p = dict(g.CONFIGS[3])
        p.update(n_r=12, n_ang=38, n_gauss=8)
        w = g.make_workload(xyz, p, 3, 200 + k, n_occ=2 * len(xyz))
        s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
        structs.append((w, s))
    yield nao, ctx, structs, torch
    for w, s in structs:
        s.close()
    ctx.close()


def _tensors(torch, w, s):
    dev = "cuda"
    return (torch.from_numpy(w["v"]).to(dev), torch.from_numpy(w["D"]).to(dev),
            torch.zeros((s.n_basis, s.n_basis), dtype=torch.float64, device=dev),
            torch.zeros(s.n_points, dtype=torch.float64, device=dev))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("capture", [False, True])
def test_many_equals_solo(env, prec, capture):
    nao, ctx, structs, torch = env
    say("run_many", prec, "capture", capture)
    tens = [_tensors(torch, w, s) for w, s in structs]
    work = []
    for (w, s), (v, D, H, n) in zip(structs, tens):
        work += [(s, "h", v, H), (s, "n", D, n)]
    ctx.run_many(work, precision=prec, capture_graph=capture)
    ctx.synchronize()
    tol = 1e-12 if prec == "fp64" else 1e-6
    for (w, s), (v, D, H, n) in zip(structs, tens):
        Hs = s.integrate_h(w["v"], precision=prec)
        ns = s.update_density(w["D"], precision=prec)
        assert rel_max(H.cpu().numpy(), Hs) <= tol
        assert rel_max(n.cpu().numpy(), ns) <= tol
        assert np.array_equal(H.cpu().numpy(), H.cpu().numpy().T)


def test_graph_replays_match_eager(env):
    nao, ctx, structs, torch = env
    say("graph replays")
    tens = [_tensors(torch, w, s) for w, s in structs]
    work = []
    for (w, s), (v, D, H, n) in zip(structs, tens):
        work += [(s, "h", v, H), (s, "n", D, n)]
    ctx.run_many(work, capture_graph=False)
    ctx.synchronize()
    eager = [(H.cpu().numpy().copy(), n.cpu().numpy().copy()) for v, D, H, n in tens]
    for rep in range(4):
        for v, D, H, n in tens:      # the program's own work between replays
            H.fill_(7.0)
            n.fill_(-3.0)
        torch.cuda.synchronize()
        ctx.run_many(work, capture_graph=True)
        ctx.synchronize()
        for (He, ne), (v, D, H, n) in zip(eager, tens):
            assert rel_max(H.cpu().numpy(), He) <= 1e-12, rep
            assert rel_max(n.cpu().numpy(), ne) <= 1e-12, rep


def test_many_matches_oracle_member(env):
    """A known case mixed with other structures still matches the oracle."""
    nao, ctx, structs, torch = env
    w1, B, ref = case("multitile")
    say("run_many oracle member")
    s1 = nao.build_batches(ctx, w1["basis"], w1["xyz"], w1["w"], w1["max_batch"])
    v1, D1, H1, n1 = _tensors(torch, w1, s1)
    work = [(s1, "h", v1, H1), (s1, "n", D1, n1)]
    for (w, s) in structs[:3]:
        v, D, H, n = _tensors(torch, w, s)
        work += [(s, "n", D, n), (s, "h", v, H)]
    ctx.run_many(work, capture_graph=True)
    ctx.synchronize()
    assert rel_max(H1.cpu().numpy(), ref["H"]) <= 1e-12
    assert rel_max(n1.cpu().numpy(), ref["n"]) <= 1e-12
    s1.close()


def test_many_with_wide_tiles(env):
    """Systems with 64- and 128-wide Hamiltonian tiles in one launch sequence."""
    nao, ctx, structs, torch = env
    say("run_many wide tiles")
    structs[1][1].set_h_tile(128)
    structs[3][1].set_h_tile(128)
    tens = [_tensors(torch, w, s) for w, s in structs]
    work = [(s, "h", v, H) for (w, s), (v, D, H, n) in zip(structs, tens)]
    ctx.run_many(work, capture_graph=True)
    ctx.synchronize()
    for (w, s), (v, D, H, n) in zip(structs, tens):
        assert rel_max(H.cpu().numpy(), s.integrate_h(w["v"])) <= 1e-12
    structs[1][1].set_h_tile(64)
    structs[3][1].set_h_tile(64)


def test_graph_dropped_when_scratch_grows():
    """A captured launch plan holds the address of the context's basis scratch.  Building a
    system with larger blocks on the same context replaces that scratch; a later replay of the
    same argument set must run a fresh capture (results equal the oracle), not the old graph."""
    import torch
    from paper_1912_06636_amd import nao
    say("graph after scratch growth")
    ctx = nao.Context(0)
    w1, B1, ref1 = case("config1")
    s1 = nao.build_batches(ctx, w1["basis"], w1["xyz"], w1["w"], w1["max_batch"])
    v1, D1, H1, n1 = _tensors(torch, w1, s1)
    work = [(s1, "h", v1, H1), (s1, "n", D1, n1)]
    ctx.run_many(work, capture_graph=True)
    ctx.synchronize()
    assert rel_max(H1.cpu().numpy(), ref1["H"]) <= 1e-12
    used0, _ = ctx.memory()
    w2, B2, ref2 = case("multitile")     # larger basis blocks: the scratch is reallocated
    s2 = nao.build_batches(ctx, w2["basis"], w2["xyz"], w2["w"], w2["max_batch"])
    for rep in range(3):
        H1.fill_(5.0)
        n1.fill_(-1.0)
        torch.cuda.synchronize()
        ctx.run_many(work, capture_graph=True)
        ctx.synchronize()
        assert rel_max(H1.cpu().numpy(), ref1["H"]) <= 1e-12, rep
        assert rel_max(n1.cpu().numpy(), ref1["n"]) <= 1e-12, rep
    # the larger system's own results stay exact, alone and together with the first
    v2, D2, H2, n2 = _tensors(torch, w2, s2)
    ctx.run_many(work + [(s2, "h", v2, H2), (s2, "n", D2, n2)], capture_graph=True)
    ctx.synchronize()
    assert rel_max(H2.cpu().numpy(), ref2["H"]) <= 1e-12 and rel_max(n2.cpu().numpy(), ref2["n"]) <= 1e-12
    assert rel_max(H1.cpu().numpy(), ref1["H"]) <= 1e-12
    assert used0 > 0
    s2.close()
    s1.close()
    ctx.close()


def test_many_on_a_caller_stream_with_electron_counts(env):
    """hip_stream and per-entry n_electrons: the work runs on the caller's stream, after the
    context's earlier work; N_e of every density entry equals the single-call value."""
    nao, ctx, structs, torch = env
    say("run_many on a caller stream with electron counts")
    tens = [_tensors(torch, w, s) for w, s in structs]
    work = []
    for (w, s), (v, D, H, n) in zip(structs, tens):
        work += [(s, "n", D, n), (s, "h", v, H)]
    st = torch.cuda.Stream()
    ne = ctx.run_many(work, stream=st.cuda_stream, electrons=True)
    assert len(ne) == len(structs)
    for (w, s), (v, D, H, n), ne_k in zip(structs, tens, ne):
        ns, Ne = s.update_density(w["D"], electrons=True)
        assert rel_max(n.cpu().numpy(), ns) <= 1e-12
        assert abs(ne_k - Ne) <= 1e-12 * abs(Ne)
        assert rel_max(H.cpu().numpy(), s.integrate_h(w["v"])) <= 1e-12
    # the context's stream orders after the caller-stream work: overwrite and rerun eagerly
    for v, D, H, n in tens:
        H.fill_(3.0)
    torch.cuda.synchronize()
    ctx.run_many([(s, "h", v, H) for (w, s), (v, D, H, n) in zip(structs, tens)], stream=st.cuda_stream)
    ctx.synchronize()
    st.synchronize()
    for (w, s), (v, D, H, n) in zip(structs, tens):
        assert rel_max(H.cpu().numpy(), s.integrate_h(w["v"])) <= 1e-12
    with pytest.raises(nao.NaoError):
        ctx.run_many(work, capture_graph=True, electrons=True)


def test_overlap_toggle_with_captured_plans(monkeypatch):
    """Chunks in two buffers with the basis launches on a second stream (blocks of at most 16 MB:
    several chunks): captured and eager results equal the oracle with the overlap on, after it is
    turned off (the second buffer is freed, so captured plans that hold it must be dropped) and
    after it is turned on again."""
    import torch
    from paper_1912_06636_amd import nao
    monkeypatch.setenv("NAO_SCRATCH_MB", "16")
    say("overlap toggle with captured plans")
    ctx = nao.Context(0)
    w1, B1, ref1 = case("multitile")
    w2, B2, ref2 = case("config1")
    s1 = nao.build_batches(ctx, w1["basis"], w1["xyz"], w1["w"], w1["max_batch"])
    s2 = nao.build_batches(ctx, w2["basis"], w2["xyz"], w2["w"], w2["max_batch"])
    t1, t2 = _tensors(torch, w1, s1), _tensors(torch, w2, s2)
    work = [(s1, "h", t1[0], t1[2]), (s1, "n", t1[1], t1[3]), (s2, "n", t2[1], t2[3]), (s2, "h", t2[0], t2[2])]
    for state in ("on", "off", "on again"):
        ctx.set_overlap(state != "off")
        for capture in (True, True, False):
            for t in (t1, t2):
                t[2].fill_(9.0)
                t[3].fill_(-9.0)
            torch.cuda.synchronize()
            ctx.run_many(work, capture_graph=capture)
            ctx.synchronize()
            for t, ref in ((t1, ref1), (t2, ref2)):
                eH, en = rel_max(t[2].cpu().numpy(), ref["H"]), rel_max(t[3].cpu().numpy(), ref["n"])
                say("overlap", state, "capture", capture, "H %.2e n %.2e" % (eH, en))
                assert eH <= 1e-12 and en <= 1e-12
    s2.close()
    s1.close()
    ctx.close()
