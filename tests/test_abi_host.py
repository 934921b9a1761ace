"""The C-ABI library on the CPU: it loads, exports every function nao.h declares, and its
host-only planning (octree batches + nnz(B) lists) is bit-exact with the oracle.  No GPU
compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis as ob
from oracle import batching as bt
from workloads import generate as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nao.h")).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(nao_\w+)\s*\(", text, flags=re.M)))


def test_header_symbols_exported():
    from paper_1912_06636_amd import nao
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(nao.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(nao.EXPORTED) == names


def test_context_without_gpu_reports_not_ready():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1912_06636_amd import nao
    with pytest.raises(nao.NaoError) as e:
        nao.Context(0)
    assert e.value.status == nao.ERR_NOT_READY


def _oracle_plan(basis, xyz, max_batch):
    B = ob.Basis(basis)
    perm, bp = bt.octree_batches(xyz, max_batch)
    lp, li = bt.basis_lists(xyz, perm, bp, B)
    return perm, bp, lp, li


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("cfg", [1, 2])
def test_plan_bit_exact_configs(cfg):
    from paper_1912_06636_amd import nao
    w = g.config_workload(cfg, with_density=False)
    assert _same(nao.plan_create(w["basis"], w["xyz"], w["max_batch"]),
                 _oracle_plan(w["basis"], w["xyz"], w["max_batch"]))


@pytest.mark.parametrize("max_batch", [1, 3, 32, 200, 4096])
def test_plan_bit_exact_two_species_and_sizes(max_batch):
    from paper_1912_06636_amd import nao
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, -0.4], [0.5, 2.1, 0.7], [3.0, 2.0, 1.0]])
    basis = g.make_basis(xyz, np.array([0, 1, 0, 1], np.int32), [(0, 1, 2, 3), (0, 0, 1)], [4.5, 3.0], 7, 0)
    X, _, _ = g.make_grid(xyz, 4.5, 10, 26)
    assert _same(nao.plan_create(basis, X, max_batch), _oracle_plan(basis, X, max_batch))


def test_plan_degenerate_points():
    from paper_1912_06636_amd import nao
    w = g.config_workload(1, with_density=False)
    xyz = np.zeros((1000, 3)) + 1.25               # coincident: chunked in index order
    xyz[500:] = 2.5
    xyz = np.concatenate([xyz, np.zeros((301, 3))])
    xyz[-1] = 9.0
    got = nao.plan_create(w["basis"], xyz, 256)
    assert _same(got, _oracle_plan(w["basis"], xyz, 256))
    # points exactly on the cutoff sphere are not relevant (strict <)
    atom0 = w["basis"]["atom_xyz"][0]
    on = np.array([atom0 + [4.0, 0.0, 0.0], atom0 + [0.0, -4.0, 0.0]])
    assert _same(nao.plan_create(w["basis"], on, 10), _oracle_plan(w["basis"], on, 10))


def test_plan_empty_and_errors():
    from paper_1912_06636_amd import nao
    w = g.config_workload(1, with_density=False)
    perm, bp, lp, li = nao.plan_create(w["basis"], np.zeros((0, 3)), 10)
    assert len(perm) == 0 and list(bp) == [0] and list(lp) == [0] and len(li) == 0
    with pytest.raises(nao.NaoError) as e:
        nao.plan_create(w["basis"], w["xyz"], 0)
    assert e.value.status == nao.ERR_INVALID_ARG
    with pytest.raises(nao.NaoError):
        nao.plan_create(w["basis"], w["xyz"], 5000)
    bad = dict(w["basis"])
    bad["shell_l"] = np.array([0, 0, 4], np.int32)
    with pytest.raises(nao.NaoError):
        nao.plan_create(bad, w["xyz"], 200)
    bad = dict(w["basis"])
    bad["radial_rcut"] = bad["radial_rmin"] * 0.5
    with pytest.raises(nao.NaoError):
        nao.plan_create(bad, w["xyz"], 200)
    xyz = w["xyz"].copy()
    xyz[5, 1] = np.nan
    with pytest.raises(nao.NaoError) as e:
        nao.plan_create(w["basis"], xyz, 200)
    assert "non-finite" in str(e.value)


def _oracle_cutplane_plan(basis, xyz, max_batch):
    B = ob.Basis(basis)
    perm, bp = bt.cutplane_batches(xyz, max_batch)
    lp, li = bt.basis_lists(xyz, perm, bp, B)
    return perm, bp, lp, li


@pytest.mark.parametrize("cfg,max_batch", [(1, 100), (1, 200), (2, 200), (2, 256)])
def test_cutplane_plan_bit_exact_configs(cfg, max_batch):
    from paper_1912_06636_amd import nao
    w = g.config_workload(cfg, with_density=False)
    got = nao.plan_create(w["basis"], w["xyz"], max_batch, batcher="cutplane")
    assert _same(got, _oracle_cutplane_plan(w["basis"], w["xyz"], max_batch))
    assert len(got[1]) - 1 == -(-len(w["xyz"]) // max_batch)


@pytest.mark.parametrize("max_batch", [1, 2, 3, 32, 4096])
def test_cutplane_bit_exact_sizes_and_degenerate_points(max_batch):
    from paper_1912_06636_amd import nao
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, -0.4], [0.5, 2.1, 0.7], [3.0, 2.0, 1.0]])
    basis = g.make_basis(xyz, np.array([0, 1, 0, 1], np.int32), [(0, 1, 2, 3), (0, 0, 1)], [4.5, 3.0], 7, 0)
    X, _, _ = g.make_grid(xyz, 4.5, 10, 26)
    assert _same(nao.plan_create(basis, X, max_batch, batcher="cutplane"),
                 _oracle_cutplane_plan(basis, X, max_batch))
    same = np.zeros((300, 3)) + 1.25                # coincident points: the index order decides
    same[150:, 2] = -0.0
    same[:150, 2] = 0.0
    assert _same(nao.plan_create(basis, same, max_batch, batcher="cutplane"),
                 _oracle_cutplane_plan(basis, same, max_batch))
    with pytest.raises(KeyError):
        nao.plan_create(basis, X, max_batch, batcher="kdtree")


def test_unknown_batcher_is_rejected():
    from paper_1912_06636_amd import nao
    w = g.config_workload(1, with_density=False)
    d = nao._Desc(w["basis"])
    xyz = np.ascontiguousarray(w["xyz"], dtype=np.float64)
    h = ctypes.c_void_p()
    st = nao._lib.nao_plan_create_ex(ctypes.byref(d.struct), len(xyz), xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     200, 7, ctypes.byref(h))
    assert st == nao.ERR_INVALID_ARG and not h.value


def test_off_chip_cases_select_their_branches():
    """The inputs of tests/test_gpu_basis_fallback.py take the branches they are meant to test:
    a spline table larger than the 8,192 doubles the basis kernel stages in LDS (and the
    two-species, 8-radial basis of a two-element slab within it), a batch (and so a unit) with
    more than the 192 atoms it stages, a system with more than the 128 shells it stages."""
    from paper_1912_06636_amd import nao
    from tests.gpu_cases import case
    for name in ("two_species_8", "dense_cluster", "many_species"):
        w, B, ref = case(name)
        b = w["basis"]
        table = len(b["radial_rmin"]) * b["n_knots"] * 2  # (y_k, M_k / 6) per knot
        n_shells = int(b["species_shell_ptr"][-1])
        perm, bp, lp, li = nao.plan_create(b, w["xyz"], w["max_batch"])
        owner = g.basis_atom_index(b)
        most_atoms = max(len(set(owner[li[lp[k]:lp[k + 1]]].tolist())) for k in range(len(lp) - 1))
        if name == "two_species_8":
            assert table <= 8192 and len(b["radial_rmin"]) == 16
        if name == "dense_cluster":
            assert most_atoms > 192
        if name == "many_species":
            assert n_shells > 128 and table > 8192
