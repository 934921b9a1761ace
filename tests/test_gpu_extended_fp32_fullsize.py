"""FP32 forms of the extended operations at full size against their FP64 forms (themselves
pinned to the oracle): density gradient, H with a vector field, H with the kinetic term and
the local Pulay forces; normwise errors printed and held to the stated FP32 bound."""
import numpy as np
import pytest

from tests.test_gpu_fullsize import full, nao, say  # noqa: F401
from workloads import generate as g

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5  # stated accuracy of the FP32 contractions of the extended operations


def rel(a, b):
    return float(np.max(np.abs(a - b))) / float(np.max(np.abs(b)))


@pytest.mark.parametrize("cfg", [2, 4])
def test_extended_operations_fp32_full_size(nao, cfg):
    say("full-size extended operations in FP32, config", cfg)
    w, B = full(cfg)
    a = 0.3 * np.random.default_rng(90 + cfg).normal(size=(len(w["xyz"]), 3))
    Q = g.energy_weighted_for(w, 1)
    ctx = nao.Context(0)
    s = nao.build_batches(ctx, w["basis"], w["xyz"], w["w"], w["max_batch"])
    errs = {}
    n64, g64 = s.update_density_gradient(w["D"])
    n32, g32 = s.update_density_gradient(w["D"], precision="fp32")
    errs["grad"] = rel(g32, g64)
    errs["gga"] = rel(s.integrate_h_gga(w["v"], a, precision="fp32"), s.integrate_h_gga(w["v"], a))
    errs["ks"] = rel(s.integrate_h_ks(w["v"], precision="fp32"), s.integrate_h_ks(w["v"]))
    errs["forces"] = rel(s.pulay_forces(w["D"], Q, w["v"], precision="fp32"), s.pulay_forces(w["D"], Q, w["v"]))
    s.close()
    ctx.close()
    say("config", cfg, " ".join("e_%s %.3e" % kv for kv in errs.items()))
    assert all(e <= FP32_TOL for e in errs.values())
