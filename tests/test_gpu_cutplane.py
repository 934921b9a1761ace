"""Cut-plane batches on the GPU: the system's batches and lists are the oracle's bit for bit,
and H and n over them match the oracle (the results do not depend on the partition), with
execution groups and with every batch its own unit."""
import sys

import numpy as np
import pytest

from oracle import batching as bt
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


@pytest.fixture(scope="module")
def ctx(nao):
    c = nao.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,max_batch", [("config1", 100), ("config1", 200), ("multitile", 200),
                                            ("two_species", 64)])
def test_cutplane_results_match_oracle(nao, ctx, name, max_batch):
    w, B, ref = case(name)
    say("cut-plane", name, max_batch)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], max_batch, batcher="cutplane")
    perm, bp, lp, li = s.get_batches()
    operm, obp = bt.cutplane_batches(w["xyz"], max_batch)
    olp, oli = bt.basis_lists(w["xyz"], operm, obp, B)
    assert np.array_equal(perm, operm) and np.array_equal(bp, obp)
    assert np.array_equal(lp, olp) and np.array_equal(li, oli)
    for gm in (256, 0):
        s.set_group_max(gm)
        H = s.integrate_h(w["v"])
        n = s.update_density(w["D"])
        eH, en = rel_max(H, ref["H"]), rel_max(n, ref["n"])
        say("cut-plane", name, max_batch, "group_max", gm, "e_H %.3e e_n %.3e" % (eH, en))
        assert eH <= 1e-12 and en <= 1e-12
    s.close()
