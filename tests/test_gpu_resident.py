"""Resident basis values (nao_system_set_resident_basis): the results equal those of the default
mode (up to the order of the FP64 atomic accumulation into H and n, which varies between runs)
through evaluation, reuse, a change of value type (FP32 and back), a change of execution groups
and switching the mode off; a budget that cannot hold the values leaves the mode off and the
system working."""
import ctypes
import sys

import numpy as np
import pytest

from tests.gpu_cases import case, rel_max

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


def results(s, w, prec):
    return s.integrate_h(w["v"], precision=prec), s.update_density(w["D"], precision=prec)


def same(got, ref, what):
    (H, n), (H0, n0) = got, ref
    eH, en = rel_max(H, H0), rel_max(n, n0)
    say(what, "e_H %.3e e_n %.3e" % (eH, en))
    assert eH <= 1e-13 and en <= 1e-13


def test_resident_basis_is_bitwise_default(nao):
    w, B, ref = case("multitile")
    say("resident basis values, multitile")
    ctx = nao.Context(0)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    r64 = results(s, w, "fp64")
    r32 = results(s, w, "fp32")
    s.set_group_max(128)
    r128 = results(s, w, "fp64")
    s.set_group_max(256)
    s.set_resident_basis(True)
    same(results(s, w, "fp64"), r64, "resident fp64, evaluated")
    same(results(s, w, "fp64"), r64, "resident fp64, reused")
    same(results(s, w, "fp32"), r32, "resident fp32")
    same(results(s, w, "fp64"), r64, "resident fp64 again")
    s.set_group_max(128)
    same(results(s, w, "fp64"), r128, "resident, groups of 128")
    same(results(s, w, "fp64"), r128, "resident, groups of 128, reused")
    s.set_resident_basis(False)
    same(results(s, w, "fp64"), r128, "mode off")
    s.close()
    ctx.close()


def test_resident_basis_over_budget_stays_off(nao):
    w, B, ref = case("multitile")
    say("resident basis values over budget")
    probe = nao.Context(0)
    s = nao.build_batches(probe, w["basis"], w["xyz"], w["w"], w["max_batch"])
    r64 = results(s, w, "fp64")
    used, budget = ctypes.c_size_t(), ctypes.c_size_t()
    assert nao._lib.nao_ctx_memory(probe.handle, ctypes.byref(used), ctypes.byref(budget)) == 0
    s.close()
    probe.close()
    ctx = nao.Context(0, hbm_budget=int(used.value) + 4096)  # the system fits, its values do not
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    same(results(s, w, "fp64"), r64, "budget-limited context")
    with pytest.raises(nao.NaoError) as e:
        s.set_resident_basis(True)
    assert e.value.status == nao.ERR_BUDGET
    same(results(s, w, "fp64"), r64, "after the refused mode")
    s.close()
    ctx.close()
