"""The density kernel with function lists longer than it stages on chip (4096 global indices):
a 150-atom cluster of 4800 functions where the units near the centre list every function, so
that the items of their last column tiles read the list from global memory while the others
read it from LDS.  FP64 and FP32 densities against the oracle, element by element, and the
many-structure launch beside a small structure."""
import sys

import numpy as np
import pytest

from tests.gpu_cases import case, rel_max, wide_list_case

pytestmark = pytest.mark.gpu
LIST_ON_CHIP = 4096


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


def test_long_lists_density(nao, ctx):
    w, B, n_ref = wide_list_case()
    say("long-list density: building batches")
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    _, _, lp, _ = s.get_batches()
    longest = int(np.max(np.diff(lp)))
    say("long-list density: longest batch list %d functions" % longest)
    assert longest > LIST_ON_CHIP
    e64 = rel_max(s.update_density(w["D"]), n_ref)
    e32 = rel_max(s.update_density(w["D"], precision="fp32"), n_ref)
    say("long-list density: fp64 %.2e fp32 %.2e" % (e64, e32))
    assert e64 <= 1e-12
    assert e32 <= 1e-5
    s.close()


def test_long_lists_many_launch(nao, ctx):
    import torch
    dev = torch.device("cuda:0")
    w, B, n_ref = wide_list_case()
    w2, _, ref2 = case("multitile")
    work, outs, systems = [], [], []
    for ww, ref in ((w, n_ref), (w2, ref2["n"])):
        s = nao.build_batches(ctx, ww["basis"], ww["xyz"], ww["w"], ww["max_batch"])
        D = torch.from_numpy(ww["D"]).to(dev)
        n = torch.empty(s.n_points, dtype=torch.float64, device=dev)
        systems.append(s)
        outs.append((D, n, ref))
        work.append((s, "n", D, n))
    torch.cuda.synchronize()
    say("long-list density: many-structure launch")
    ctx.run_many(work)
    ctx.synchronize()
    for k, (D, n, ref) in enumerate(outs):
        e = rel_max(n.cpu().numpy(), ref)
        say("long-list density: many-structure launch, structure %d: %.2e" % (k, e))
        assert e <= 1e-12
    for s in systems:
        s.close()
