"""Full-size cut-plane batches: results against the octree path and, on the block, batches and lists against the oracle."""
import numpy as np
import pytest

from tests.test_gpu_fullsize import fp64_results, full, nao, say  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [2, 4])
def test_cutplane_batches_full_size(nao, cfg):
    """Cut-plane batches of 256 at full size: the results equal those over the octree batches
    (pinned to the oracle above); on the block the batches and lists are the oracle's bit for bit."""
    say("full-size cut-plane batches, config", cfg)
    from oracle import batching as bt
    w, B = full(cfg)
    H64, _, n64, _ = fp64_results(cfg)
    ctx = nao.Context(0)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], 256, batcher="cutplane")
    assert s.n_batches == -(-len(w["xyz"]) // 256)
    if cfg == 2:
        perm, bp, lp, li = s.get_batches()
        operm, obp = bt.cutplane_batches(w["xyz"], 256)
        olp, oli = bt.basis_lists(w["xyz"], operm, obp, B)
        assert np.array_equal(perm, operm) and np.array_equal(bp, obp)
        assert np.array_equal(lp, olp) and np.array_equal(li, oli)
    H = s.integrate_h(w["v"])
    n = s.update_density(w["D"])
    s.close()
    ctx.close()
    eH = float(np.max(np.abs(H - H64))) / float(np.max(np.abs(H64)))
    en = float(np.max(np.abs(n - n64))) / float(np.max(np.abs(n64)))
    say("config", cfg, "cut-plane vs octree: e_H %.3e e_n %.3e" % (eH, en))
    assert eH <= 1e-12 and en <= 1e-12
    assert np.array_equal(H, H.T)
