"""Serving core on the GPU: served results equal the FP64 oracle's (first iteration with its
own potential, second iteration with a fresh D and the kept potential); each request's result
is the same alone and in a mix of concurrently admitted structures, in every precision;
admission respects the HBM budget (sessions wait for memory, then run); closed sessions free
their memory; a result is readable until its session's next request starts."""
import sys
import time

import numpy as np
import pytest

from oracle import basis as ob
from oracle import integrals as oi
from tests.gpu_cases import rel_max
from workloads import generate as g

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def small(k, n_atoms):
    xyz = g.geometry_sc_first_n(n_atoms, 2.2, 0.1, g.rng_for(5, 300 + k, 0))
    p = dict(g.CONFIGS[3])
    p.update(n_r=12, n_ang=38, n_gauss=8)
    return g.make_workload(xyz, p, 5, 300 + k, n_occ=2 * n_atoms)


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_06636_amd import nao
    return nao


def drain(srv, tickets, timeout=120.0):
    t0 = time.time()
    while True:
        srv.step()
        if all(srv.poll(t)[0] == 2 for t in tickets):
            return
        assert time.time() - t0 < timeout, "serving requests did not finish"
        time.sleep(0.0005)


# Stated normwise bounds against FP64 of the batched precisions (the serving default is fp32).
SERVE_TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 3e-5, "bf16x6": 1e-6}


def test_served_results_match_oracle(lib):
    """Two iterations of one session against the oracle: (D1, v) then (D2, kept v)."""
    say("serve vs oracle")
    w = small(40, 14)
    B = ob.Basis(w["basis"])
    rng = np.random.default_rng(41)
    C2 = rng.normal(size=(w["n_basis"], 20))
    D2 = C2 @ C2.T
    H_ref = oi.hamiltonian(B, w["xyz"], w["w"], w["v"])
    n1_ref = oi.density(B, w["xyz"], w["D"])
    n2_ref = oi.density(B, w["xyz"], D2)
    home = lib.Context(0)
    srv = lib.Server(home, n_slots=2, max_per_launch=4, precision="fp64")
    sid = srv.open_session(w["basis"], w["xyz"], w["w"], 256)
    nb, npt = w["n_basis"], len(w["xyz"])
    t1 = srv.submit(sid, w["D"], w["v"])
    drain(srv, [t1])
    H1, n1 = np.empty((nb, nb)), np.empty(npt)
    srv.result(t1, H1, n1)
    say("serve vs oracle", "iteration 1: e_H %.2e e_n %.2e" % (rel_max(H1, H_ref), rel_max(n1, n1_ref)))
    assert rel_max(H1, H_ref) <= 1e-12 and rel_max(n1, n1_ref) <= 1e-12
    t2 = srv.submit(sid, D2)                          # fresh D, the potential of iteration 1
    drain(srv, [t2])
    H2, n2 = np.empty((nb, nb)), np.empty(npt)
    srv.result(t2, H2, n2)
    say("serve vs oracle", "iteration 2: e_H %.2e e_n %.2e" % (rel_max(H2, H_ref), rel_max(n2, n2_ref)))
    assert rel_max(H2, H_ref) <= 1e-12 and rel_max(n2, n2_ref) <= 1e-12
    # iteration 1's result was replaced by iteration 2's: the server says so
    with pytest.raises(lib.NaoError) as e:
        srv.result(t1, H1, n1)
    assert e.value.status == lib.ERR_INVALID_ARG
    srv.close()
    home.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_alone_equals_mix(lib, prec):
    say("serve alone vs mix", prec)
    works = [small(k, n) for k, n in enumerate([9, 14, 20, 6, 12])]
    home = lib.Context(0)
    # alone: one session, one request
    srv = lib.Server(home, n_slots=1, max_per_launch=1, precision=prec)
    sid = srv.open_session(works[0]["basis"], works[0]["xyz"], works[0]["w"], 256)
    tk = srv.submit(sid, works[0]["D"], works[0]["v"])
    drain(srv, [tk])
    nb = works[0]["n_basis"]
    H_alone = np.empty((nb, nb))
    n_alone = np.empty(len(works[0]["xyz"]))
    srv.result(tk, H_alone, n_alone)
    srv.close()
    # mix: all sessions at once over three slots, several requests per launch
    srv = lib.Server(home, n_slots=3, max_per_launch=2, precision=prec)
    sids = [srv.open_session(w["basis"], w["xyz"], w["w"], 256) for w in works]
    tks = [srv.submit(s, w["D"], w["v"]) for s, w in zip(sids, works)]
    drain(srv, tks)
    H_mix = np.empty((nb, nb))
    n_mix = np.empty(len(works[0]["xyz"]))
    srv.result(tks[0], H_mix, n_mix)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert rel_max(H_mix, H_alone) <= tol and rel_max(n_mix, n_alone) <= tol
    # and against the oracle, within the precision's stated bound
    B0 = ob.Basis(works[0]["basis"])
    eH = rel_max(H_mix, oi.hamiltonian(B0, works[0]["xyz"], works[0]["w"], works[0]["v"]))
    en = rel_max(n_mix, oi.density(B0, works[0]["xyz"], works[0]["D"]))
    say("serve alone vs mix", prec, "vs oracle: e_H %.2e e_n %.2e" % (eH, en))
    assert eH <= SERVE_TOL[prec] and en <= SERVE_TOL[prec]
    # the other members against their own single-call results
    for s, w, t in zip(sids[1:], works[1:], tks[1:]):
        sysm = lib.build_batches(home, w["basis"], w["xyz"], w["w"], 256)
        Hs = sysm.integrate_h(w["v"], precision=prec)
        ns = sysm.update_density(w["D"], precision=prec)
        Hm = np.empty_like(Hs)
        nm = np.empty_like(ns)
        srv.result(t, Hm, nm)
        assert rel_max(Hm, Hs) <= tol and rel_max(nm, ns) <= tol
        sysm.close()
    srv.close()
    home.close()


def test_admission_by_budget_and_iterations(lib):
    say("serve admission")
    works = [small(10 + k, n) for k, n in enumerate([12, 12, 12])]
    probe = lib.Context(0)
    s0 = lib.Server(probe, n_slots=1, max_per_launch=1)
    sid = s0.open_session(works[0]["basis"], works[0]["xyz"], works[0]["w"], 256)
    one = s0.wait_settled(sid)["bytes"]
    used_before, _ = probe.memory()
    s0.close()
    probe.close()
    assert one > 0
    # room for the first session (plus the context's own buffers) and half of another one
    home = lib.Context(0, hbm_budget=int(used_before + one // 2))
    srv = lib.Server(home, n_slots=2, max_per_launch=4)
    sids = [srv.open_session(w["basis"], w["xyz"], w["w"], 256) for w in works]
    assert srv.wait_settled(sids[0])["state"] == lib.SESSION_RESIDENT
    assert srv.wait_settled(sids[1])["state"] == lib.SESSION_NO_MEMORY
    assert srv.session_info(sids[2])["state"] in (lib.SESSION_QUEUED, lib.SESSION_NO_MEMORY)  # behind sids[1]
    # two iterations on the first session, then close it: the next one gets admitted
    t1 = srv.submit(sids[0], works[0]["D"], works[0]["v"])
    t2 = srv.submit(sids[0], works[0]["D"])          # keeps the previous v
    t3 = srv.submit(sids[1], works[1]["D"], works[1]["v"])
    drain(srv, [t1, t2])
    st1, st2 = srv.poll(t1), srv.poll(t2)
    assert st1[3] <= st2[2] + 1e-9                    # iterations of one session run in order
    assert srv.poll(t3)[0] == 0                       # still waiting for memory
    H0 = np.empty((works[0]["n_basis"],) * 2)
    with pytest.raises(lib.NaoError):                 # t2 replaced t1's result
        srv.result(t1, H0)
    srv.result(t2, H0)
    B0 = ob.Basis(works[0]["basis"])
    assert rel_max(H0, oi.hamiltonian(B0, works[0]["xyz"], works[0]["w"], works[0]["v"])) <= 1e-12
    srv.close_session(sids[0])
    drain(srv, [t3])
    assert srv.session_info(sids[1])["resident"]
    assert srv.session_info(sids[0])["state"] == lib.SESSION_CLOSED
    H = np.empty((works[1]["n_basis"],) * 2)
    srv.result(t3, H)
    other = lib.Context(0)                            # the home context has no room left
    sysm = lib.build_batches(other, works[1]["basis"], works[1]["xyz"], works[1]["w"], 256)
    assert rel_max(H, sysm.integrate_h(works[1]["v"])) <= 1e-12
    sysm.close()
    other.close()
    srv.close()
    home.close()


def test_session_larger_than_budget_fails(lib):
    say("serve oversize session")
    w = small(20, 12)
    home = lib.Context(0, hbm_budget=1 << 20)
    srv = lib.Server(home, n_slots=1, max_per_launch=1)
    sid = srv.open_session(w["basis"], w["xyz"], w["w"], 256)
    try:
        tk = srv.submit(sid, w["D"], w["v"])
    except lib.NaoError:
        tk = None                                     # the builder was quicker: already failed
    assert srv.wait_settled(sid)["state"] == lib.SESSION_FAILED
    if tk is not None:
        assert srv.poll(tk)[0] == lib.REQ_FAILED
    srv.close()
    home.close()
