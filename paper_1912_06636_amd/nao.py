"""Thin ctypes binding of libnao.so (include/nao.h): argument marshalling only.

Every step of the grid operations runs inside the HIP library; this module converts
numpy arrays / torch tensors to pointers and status codes to exceptions.  Device
memory comes from torch (``tensor.data_ptr()`` with memspace DEVICE); host arrays are
numpy (memspace HOST).  There is no fallback: if libnao.so is missing or cannot load,
importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
import time
import weakref

import numpy as np

try:  # load torch first so that libnao.so binds to the HIP runtime torch already uses
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for the host-only planning calls
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnao.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libnao.so is not built; run `python -m paper_1912_06636_amd.build` "
                      "(the grid operations have no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_BUDGET, ERR_HIP, ERR_NOT_READY, ERR_INTERNAL = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
MEM_HOST, MEM_DEVICE = 0, 1
RUN_CAPTURE_GRAPH = 1

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class BasisDesc(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int64), ("atom_xyz", _c_dp), ("atom_species", _c_i32p),
        ("n_species", ctypes.c_int32), ("species_shell_ptr", _c_i32p), ("shell_l", _c_i32p),
        ("shell_radial", _c_i32p), ("n_radial", ctypes.c_int32), ("n_knots", ctypes.c_int32),
        ("radial_rmin", _c_dp), ("radial_rcut", _c_dp), ("radial_samples", _c_dp),
    ]


class Work(ctypes.Structure):
    _fields_ = [("sys", _vp), ("op", ctypes.c_int32), ("input", _vp), ("output", _vp), ("n_electrons", _c_dp)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_S = ctypes.c_int
_sig("nao_ctx_create", _S, ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(_vp))
_sig("nao_ctx_destroy", None, _vp)
_sig("nao_last_error", ctypes.c_char_p, _vp)
_sig("nao_ctx_set_stream", _S, _vp, _vp)
_sig("nao_ctx_stream", _vp, _vp)
_sig("nao_ctx_synchronize", _S, _vp)
_sig("nao_ctx_memory", _S, _vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t))
_sig("nao_ctx_set_overlap", _S, _vp, ctypes.c_int)
_sig("nao_ctx_profile", _S, _vp, ctypes.c_int)
_sig("nao_ctx_profile_read", _S, _vp, ctypes.c_int32, ctypes.c_char_p, _c_i64p, _c_dp, _c_i32p)
_sig("nao_plan_create", _S, ctypes.POINTER(BasisDesc), ctypes.c_int64, _c_dp, ctypes.c_int32, ctypes.POINTER(_vp))
_sig("nao_plan_create_ex", _S, ctypes.POINTER(BasisDesc), ctypes.c_int64, _c_dp, ctypes.c_int32, ctypes.c_int,
     ctypes.POINTER(_vp))
_sig("nao_plan_info", _S, _vp, _c_i64p, _c_i64p, _c_i64p)
_sig("nao_plan_get_batches", _S, _vp, _c_i64p, _c_i64p, _c_i64p, _c_i32p)
_sig("nao_plan_destroy", None, _vp)
_sig("nao_build_batches", _S, _vp, ctypes.POINTER(BasisDesc), ctypes.c_int64, _c_dp, _c_dp, ctypes.c_int32,
     ctypes.POINTER(_vp))
_sig("nao_build_batches_ex", _S, _vp, ctypes.POINTER(BasisDesc), ctypes.c_int64, _c_dp, _c_dp, ctypes.c_int32,
     ctypes.c_int, ctypes.POINTER(_vp))
_sig("nao_system_set_group_max", _S, _vp, ctypes.c_int32)
_sig("nao_system_set_resident_basis", _S, _vp, ctypes.c_int)
_sig("nao_system_set_h_tile", _S, _vp, ctypes.c_int32)
_sig("nao_system_autotune", _S, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_uint32, _c_i32p, _c_i32p, _c_dp)
_sig("nao_system_info", _S, _vp, _c_i64p, _c_i64p, _c_i64p, ctypes.POINTER(ctypes.c_size_t))
_sig("nao_get_batches", _S, _vp, _c_i64p, _c_i64p, _c_i64p, _c_i32p)
_sig("nao_system_work", _S, _vp, _c_dp)
_sig("nao_eval_basis", _S, _vp, ctypes.c_int64, ctypes.c_int64, _vp, ctypes.c_int, _c_i64p)
_sig("nao_integrate_h", _S, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int)
_sig("nao_integrate_h_noalloc", _S, _vp, _vp, ctypes.c_int, _vp)
_sig("nao_update_density", _S, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _c_dp)
_sig("nao_update_density_gradient", _S, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int)
_sig("nao_pulay_forces", _S, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int)
_sig("nao_integrate_h_ks", _S, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int)
_sig("nao_integrate_h_gga", _S, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int)
_sig("nao_system_destroy", None, _vp)
_sig("nao_run_many", _S, _vp, ctypes.POINTER(Work), ctypes.c_int64, ctypes.c_int, _vp, ctypes.c_uint32)
_sig("nao_server_create", _S, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(_vp))
_sig("nao_server_open_session", _S, _vp, ctypes.POINTER(BasisDesc), ctypes.c_int64, _c_dp, _c_dp, ctypes.c_int32,
     _c_i64p)
_sig("nao_server_close_session", _S, _vp, ctypes.c_int64)
_sig("nao_server_session_info", _S, _vp, ctypes.c_int64, _c_i32p, ctypes.POINTER(ctypes.c_size_t), _c_i64p, _c_i64p)
_sig("nao_server_submit", _S, _vp, ctypes.c_int64, _vp, ctypes.c_int, _vp, ctypes.c_int,
     ctypes.POINTER(ctypes.c_uint64))
_sig("nao_server_step", _S, _vp, _c_i32p, _c_i32p)
_sig("nao_server_poll", _S, _vp, ctypes.c_uint64, _c_i32p, _c_dp, _c_dp, _c_dp)
_sig("nao_server_result", _S, _vp, ctypes.c_uint64, _vp, _vp, ctypes.c_int)
_sig("nao_server_destroy", None, _vp)

EXPORTED = [
    "nao_ctx_create", "nao_ctx_destroy", "nao_last_error", "nao_ctx_set_stream", "nao_ctx_stream",
    "nao_ctx_synchronize", "nao_ctx_memory", "nao_ctx_set_overlap", "nao_ctx_profile", "nao_ctx_profile_read", "nao_plan_create", "nao_plan_info", "nao_plan_get_batches",
    "nao_plan_destroy", "nao_build_batches", "nao_system_set_group_max", "nao_system_set_h_tile", "nao_system_autotune", "nao_system_info", "nao_get_batches",
    "nao_system_work", "nao_eval_basis", "nao_integrate_h", "nao_update_density", "nao_update_density_gradient", "nao_integrate_h_gga",
    "nao_pulay_forces", "nao_integrate_h_ks", "nao_plan_create_ex", "nao_build_batches_ex",
    "nao_system_set_resident_basis", "nao_integrate_h_noalloc",
    "nao_system_destroy",
    "nao_run_many", "nao_server_create", "nao_server_open_session", "nao_server_close_session",
    "nao_server_session_info", "nao_server_submit", "nao_server_step", "nao_server_poll", "nao_server_result",
    "nao_server_destroy",
]


class NaoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("nao status %d: %s" % (status, msg))
        self.status = status


def _check(status, ctx=None):
    if status != OK:
        msg = _lib.nao_last_error(ctx)
        raise NaoError(status, msg.decode() if msg else "")


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t):
    return a.ctypes.data_as(t)


class _Desc:
    """Keeps the arrays of a basis description alive next to its ctypes struct."""

    def __init__(self, basis):
        self.arrays = dict(
            atom_xyz=_f64(basis["atom_xyz"]).reshape(-1, 3), atom_species=_i32(basis["atom_species"]),
            species_shell_ptr=_i32(basis["species_shell_ptr"]), shell_l=_i32(basis["shell_l"]),
            shell_radial=_i32(basis["shell_radial"]), radial_rmin=_f64(basis["radial_rmin"]),
            radial_rcut=_f64(basis["radial_rcut"]), radial_samples=_f64(basis["radial_samples"]))
        a = self.arrays
        n_knots = int(basis.get("n_knots", a["radial_samples"].shape[-1]))
        self.struct = BasisDesc(
            len(a["atom_xyz"]), _p(a["atom_xyz"], _c_dp), _p(a["atom_species"], _c_i32p),
            len(a["species_shell_ptr"]) - 1, _p(a["species_shell_ptr"], _c_i32p), _p(a["shell_l"], _c_i32p),
            _p(a["shell_radial"], _c_i32p), len(a["radial_rmin"]), n_knots, _p(a["radial_rmin"], _c_dp),
            _p(a["radial_rcut"], _c_dp), _p(a["radial_samples"], _c_dp))


def _ptr_space(x):
    """(pointer, memspace, keepalive) of a numpy array or torch tensor."""
    if torch is not None and isinstance(x, torch.Tensor):
        if x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("tensors must be contiguous float64")
        if x.is_cuda:
            return ctypes.c_void_p(x.data_ptr()), MEM_DEVICE, x
        x = x.numpy()
    if not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.flags.c_contiguous):
        raise ValueError("host arrays must be C-contiguous float64 numpy arrays")
    return ctypes.c_void_p(x.ctypes.data), MEM_HOST, x


# ---------------------------------------------------------------------------------------------
# host-only planning

BATCHERS = {"octree": 0, "cutplane": 1}


def plan_create(basis, xyz, max_batch, batcher="octree"):
    """nao_plan_create_ex + nao_plan_get_batches: (perm, batch_ptr, basis_ptr, basis_idx)."""
    d = _Desc(basis)
    xyz = _f64(xyz).reshape(-1, 3)
    h = _vp()
    _check(_lib.nao_plan_create_ex(ctypes.byref(d.struct), len(xyz), _p(xyz, _c_dp), int(max_batch),
                                   BATCHERS[batcher], ctypes.byref(h)))
    try:
        nbas, nb, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.nao_plan_info(h, ctypes.byref(nbas), ctypes.byref(nb), ctypes.byref(nl)))
        perm = np.empty(len(xyz), np.int64)
        bp = np.empty(nb.value + 1, np.int64)
        lp = np.empty(nb.value + 1, np.int64)
        li = np.empty(nl.value, np.int32)
        _check(_lib.nao_plan_get_batches(h, _p(perm, _c_i64p), _p(bp, _c_i64p), _p(lp, _c_i64p), _p(li, _c_i32p)))
        return perm, bp, lp, li
    finally:
        _lib.nao_plan_destroy(h)


# ---------------------------------------------------------------------------------------------
# context and systems

class Context:
    """nao_ctx: one device, one stream, an HBM budget (0 = none)."""

    def __init__(self, device=0, stream=None, hbm_budget=0):
        h = _vp()
        st = 0 if stream is None else int(stream)
        _check(_lib.nao_ctx_create(int(device), _vp(st) if st else None, int(hbm_budget), ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._children = weakref.WeakSet()  # systems and servers: destroyed before the context

    def close(self):
        if self.handle:
            for ch in list(self._children):
                ch.close()
            _lib.nao_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        msg = _lib.nao_last_error(self.handle)
        return msg.decode() if msg else ""

    def synchronize(self):
        _check(_lib.nao_ctx_synchronize(self.handle), self.handle)

    def set_stream(self, stream):
        _check(_lib.nao_ctx_set_stream(self.handle, _vp(int(stream)) if stream else None), self.handle)

    @property
    def stream(self):
        return _lib.nao_ctx_stream(self.handle)

    def memory(self):
        u, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.nao_ctx_memory(self.handle, ctypes.byref(u), ctypes.byref(b)), self.handle)
        return u.value, b.value

    def set_overlap(self, enable=True):
        """nao_ctx_set_overlap: basis evaluation of the next block beside the current contraction."""
        _check(_lib.nao_ctx_set_overlap(self.handle, 1 if enable else 0), self.handle)

    def profile(self, enable=True):
        _check(_lib.nao_ctx_profile(self.handle, 1 if enable else 0), self.handle)

    def profile_read(self):
        """{kernel name: (launches, total ms)} recorded since profiling was enabled."""
        cap = 64
        names = ctypes.create_string_buffer(32 * cap)
        cnt = np.zeros(cap, np.int64)
        ms = np.zeros(cap, np.float64)
        n = ctypes.c_int32()
        _check(_lib.nao_ctx_profile_read(self.handle, cap, names, _p(cnt, _c_i64p), _p(ms, _c_dp),
                                         ctypes.byref(n)), self.handle)
        raw = names.raw
        out = {}
        for k in range(min(n.value, cap)):
            nm = raw[32 * k:32 * (k + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (int(cnt[k]), float(ms[k]))
        return out

    def run_many(self, work, precision="fp64", capture_graph=False, stream=None, electrons=False):
        """nao_run_many over [(system, op, input_tensor, output_tensor)], op 'h' or 'n'.  stream: a
        hipStream_t (int) to run on instead of the context's.  electrons=True returns N_e of every
        density entry (in work order) and synchronizes."""
        arr = (Work * len(work))()
        keep = []
        ne = np.zeros(len(work), np.float64)
        for k, (sys_, op, x, y) in enumerate(work):
            px, sx, kx = _ptr_space(x)
            py, sy, ky = _ptr_space(y)
            if sx != MEM_DEVICE or sy != MEM_DEVICE:
                raise ValueError("run_many takes device tensors only")
            keep += [kx, ky]
            pe = ne[k:].ctypes.data_as(_c_dp) if electrons and op == "n" else None
            arr[k] = Work(sys_.handle, 0 if op == "h" else 1, px, py, pe)
        _check(_lib.nao_run_many(self.handle, arr, len(work), PRECISIONS[precision],
                                 _vp(stream) if stream else None,
                                 RUN_CAPTURE_GRAPH if capture_graph else 0), self.handle)
        if electrons:
            return [float(ne[k]) for k, wk in enumerate(work) if wk[1] == "n"]


def build_batches(ctx, basis, xyz, w, max_batch, batcher="octree"):
    """nao_build_batches_ex: resident device state of one structure."""
    return System(ctx, basis, xyz, w, max_batch, batcher)


class System:
    def __init__(self, ctx, basis, xyz, w, max_batch, batcher="octree"):
        d = _Desc(basis)
        xyz = _f64(xyz).reshape(-1, 3)
        w = _f64(w)
        h = _vp()
        _check(_lib.nao_build_batches_ex(ctx.handle, ctypes.byref(d.struct), len(xyz), _p(xyz, _c_dp), _p(w, _c_dp),
                                         int(max_batch), BATCHERS[batcher], ctypes.byref(h)), ctx.handle)
        self.ctx = ctx
        self.handle = h
        ctx._children.add(self)
        self.n_points = len(xyz)
        self.n_atoms = int(d.struct.n_atoms)
        info = self.info()
        self.n_basis, self.n_batches, self.n_list = info[0], info[1], info[2]

    def close(self):
        if self.handle:
            if self.ctx.handle:
                _lib.nao_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(_lib.nao_system_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
               self.ctx.handle)
        return a.value, b.value, c.value, d.value

    def set_group_max(self, g):
        _check(_lib.nao_system_set_group_max(self.handle, int(g)), self.ctx.handle)

    def set_resident_basis(self, enable=True):
        """nao_system_set_resident_basis: keep the basis values resident across operations."""
        _check(_lib.nao_system_set_resident_basis(self.handle, 1 if enable else 0), self.ctx.handle)

    def set_h_tile(self, t):
        _check(_lib.nao_system_set_h_tile(self.handle, int(t)), self.ctx.handle)

    def autotune(self, v, D, precision="fp64", force=False):
        """nao_system_autotune: returns (h_tile, group_max, best_ms or -1 if cached)."""
        pv, sv, kv = _ptr_space(v)
        pd, sd, kd = _ptr_space(D)
        if sv != sd:
            raise ValueError("v and D must be in the same memory space")
        ht, gm, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(_lib.nao_system_autotune(self.handle, PRECISIONS[precision], pv, pd, sv, 1 if force else 0,
                                        ctypes.byref(ht), ctypes.byref(gm), ctypes.byref(ms)), self.ctx.handle)
        return ht.value, gm.value, ms.value

    def work_units(self):
        u = ctypes.c_double()
        _check(_lib.nao_system_work(self.handle, ctypes.byref(u)), self.ctx.handle)
        return u.value

    def get_batches(self):
        """nao_get_batches: (perm, batch_ptr, basis_ptr, basis_idx)."""
        perm = np.empty(self.n_points, np.int64)
        bp = np.empty(self.n_batches + 1, np.int64)
        lp = np.empty(self.n_batches + 1, np.int64)
        li = np.empty(self.n_list, np.int32)
        _check(_lib.nao_get_batches(self.handle, _p(perm, _c_i64p), _p(bp, _c_i64p), _p(lp, _c_i64p),
                                    _p(li, _c_i32p)), self.ctx.handle)
        return perm, bp, lp, li

    def eval_basis(self, batch_begin=0, batch_end=None, out=None):
        """nao_eval_basis: (phi, phi_ptr); phi concatenates per-batch [|B|][m] blocks."""
        if batch_end is None:
            batch_end = self.n_batches
        ptr = np.empty(batch_end - batch_begin + 1, np.int64)
        _check(_lib.nao_eval_basis(self.handle, batch_begin, batch_end, None, MEM_HOST, _p(ptr, _c_i64p)),
               self.ctx.handle)
        if out is None:
            out = np.empty(int(ptr[-1]), np.float64)
        po, so, keep = _ptr_space(out)
        _check(_lib.nao_eval_basis(self.handle, batch_begin, batch_end, po, so, _p(ptr, _c_i64p)), self.ctx.handle)
        return out, ptr

    def integrate_h(self, v, precision="fp64", out=None):
        """nao_integrate_h: H (numpy if v is host and out is None, else into out)."""
        pv, sv, kv = _ptr_space(v)
        if out is None:
            out = np.empty((self.n_basis, self.n_basis), np.float64)
        ph, sh, kh = _ptr_space(out)
        _check(_lib.nao_integrate_h(self.handle, pv, sv, PRECISIONS[precision], ph, sh), self.ctx.handle)
        return out

    def integrate_h_noalloc(self, v, out, precision="fp64"):
        """nao_integrate_h_noalloc: H into out; v and out must be device tensors."""
        pv, sv, kv = _ptr_space(v)
        ph, sh, kh = _ptr_space(out)
        if sv != MEM_DEVICE or sh != MEM_DEVICE:
            raise ValueError("nao_integrate_h_noalloc takes device memory only")
        _check(_lib.nao_integrate_h_noalloc(self.handle, pv, PRECISIONS[precision], ph), self.ctx.handle)
        return out

    def update_density(self, D, precision="fp64", out=None, electrons=False):
        """nao_update_density: n (and N_e if electrons=True)."""
        pd, sd, kd = _ptr_space(D)
        if out is None:
            out = np.empty(self.n_points, np.float64)
        pn, sn, kn = _ptr_space(out)
        ne = ctypes.c_double(0.0)
        _check(_lib.nao_update_density(self.handle, pd, sd, PRECISIONS[precision], pn, sn,
                                       ctypes.byref(ne) if electrons else None), self.ctx.handle)
        return (out, ne.value) if electrons else out

    def integrate_h_gga(self, v, a, precision="fp64", out=None):
        """nao_integrate_h_gga: H with the local potential v and the vector field a [n_points, 3]."""
        pv, sv, kv = _ptr_space(v)
        pa, sa, ka = _ptr_space(a)
        if sv != sa:
            raise ValueError("v and a must be in the same memory space")
        if out is None:
            out = np.empty((self.n_basis, self.n_basis), np.float64)
        ph, sh, kh = _ptr_space(out)
        _check(_lib.nao_integrate_h_gga(self.handle, pv, pa, sv, PRECISIONS[precision], ph, sh), self.ctx.handle)
        return out

    def integrate_h_ks(self, v, a=None, precision="fp64", out=None):
        """nao_integrate_h_ks: H with the kinetic term, the local potential v and (a not None)
        the vector field a [n_points, 3]."""
        pv, sv, kv = _ptr_space(v)
        pa, sa = None, sv
        if a is not None:
            pa, sa, ka = _ptr_space(a)
        if sv != sa:
            raise ValueError("v and a must be in the same memory space")
        if out is None:
            out = np.empty((self.n_basis, self.n_basis), np.float64)
        ph, sh, kh = _ptr_space(out)
        _check(_lib.nao_integrate_h_ks(self.handle, pv, pa, sv, PRECISIONS[precision], ph, sh), self.ctx.handle)
        return out

    def update_density_gradient(self, D, precision="fp64", out=None, out_grad=None):
        """nao_update_density_gradient: (n, grad n [n_points, 3]); outputs share a memory space."""
        pd, sd, kd = _ptr_space(D)
        if out is None:
            out = np.empty(self.n_points, np.float64)
        if out_grad is None:
            out_grad = np.empty((self.n_points, 3), np.float64)
        pn, sn, kn = _ptr_space(out)
        pg, sg, kg = _ptr_space(out_grad)
        if sn != sg:
            raise ValueError("n and grad_n must be in the same memory space")
        _check(_lib.nao_update_density_gradient(self.handle, pd, sd, PRECISIONS[precision], pn, pg, sn),
               self.ctx.handle)
        return out, out_grad

    def pulay_forces(self, D, Q, v, precision="fp64", out=None):
        """nao_pulay_forces: local Pulay forces [n_atoms, 3]; D, Q and v share a memory space."""
        pd, sd, kd = _ptr_space(D)
        pq, sq, kq = _ptr_space(Q)
        pv, sv, kv = _ptr_space(v)
        if not (sd == sq == sv):
            raise ValueError("D, Q and v must be in the same memory space")
        if out is None:
            out = np.empty((self.n_atoms, 3), np.float64)
        pf, sf, kf = _ptr_space(out)
        _check(_lib.nao_pulay_forces(self.handle, pd, pq, pv, sd, PRECISIONS[precision], pf, sf), self.ctx.handle)
        return out


# ---------------------------------------------------------------------------------------------
# serving core

REQ_WAITING, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
SESSION_QUEUED, SESSION_RESIDENT, SESSION_NO_MEMORY, SESSION_CLOSED, SESSION_FAILED = 0, 1, 2, 3, 4


class Server:
    """nao_server: sessions admitted by the home context's HBM budget, n_slots stream slots,
    continuous batching of (density, Hamiltonian) iteration requests."""

    def __init__(self, home, n_slots=2, max_per_launch=8, precision="fp64", group_max=256):
        h = _vp()
        _check(_lib.nao_server_create(home.handle, int(n_slots), int(max_per_launch), int(group_max),
                                      PRECISIONS[precision], ctypes.byref(h)), home.handle)
        self.home = home
        self.handle = h
        self._keep = {}
        home._children.add(self)

    def close(self):
        if self.handle:
            if self.home.handle:
                _lib.nao_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open_session(self, basis, xyz, w, max_batch):
        d = _Desc(basis)
        xyz = _f64(xyz).reshape(-1, 3)
        w = _f64(w)
        sid = ctypes.c_int64()
        _check(_lib.nao_server_open_session(self.handle, ctypes.byref(d.struct), len(xyz), _p(xyz, _c_dp),
                                            _p(w, _c_dp), int(max_batch), ctypes.byref(sid)), self.home.handle)
        return sid.value

    def close_session(self, sid):
        _check(_lib.nao_server_close_session(self.handle, int(sid)), self.home.handle)

    def session_info(self, sid):
        r, b, nb, npt = ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.nao_server_session_info(self.handle, int(sid), ctypes.byref(r), ctypes.byref(b), ctypes.byref(nb),
                                            ctypes.byref(npt)), self.home.handle)
        return dict(state=r.value, resident=r.value == SESSION_RESIDENT, bytes=b.value, n_basis=nb.value,
                    n_points=npt.value)

    def wait_settled(self, sid, timeout=60.0):
        """Step the server until the session is resident, out of memory, closed or failed."""
        t0 = time.monotonic()
        while True:
            self.step()
            info = self.session_info(sid)
            if info["state"] != SESSION_QUEUED:
                return info
            if time.monotonic() - t0 > timeout:
                raise TimeoutError("session %d not admitted within %.0f s" % (sid, timeout))
            time.sleep(0.0005)

    def submit(self, sid, D, v=None):
        """Queue one iteration; D (and v) must stay valid until the request is done."""
        pd, sd, kd = _ptr_space(D)
        if v is not None:
            pv, sv, kv = _ptr_space(v)
        else:
            pv, sv, kv = None, MEM_HOST, None
        tk = ctypes.c_uint64()
        _check(_lib.nao_server_submit(self.handle, int(sid), pd, sd, pv, sv, ctypes.byref(tk)), self.home.handle)
        self._keep[tk.value] = (kd, kv)
        return tk.value

    def step(self):
        r, w = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.nao_server_step(self.handle, ctypes.byref(r), ctypes.byref(w)), self.home.handle)
        return r.value, w.value

    def poll(self, ticket):
        st = ctypes.c_int32()
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.nao_server_poll(self.handle, int(ticket), ctypes.byref(st), ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)), self.home.handle)
        if st.value in (REQ_DONE, REQ_FAILED):
            self._keep.pop(int(ticket), None)
        return st.value, a.value, b.value, c.value

    def result(self, ticket, H=None, n=None):
        ph, sh, kh = _ptr_space(H) if H is not None else (None, MEM_HOST, None)
        pn, sn, kn = _ptr_space(n) if n is not None else (None, sh, None)
        if H is not None and n is not None and sh != sn:
            raise ValueError("H and n must be in the same memory space")
        _check(_lib.nao_server_result(self.handle, int(ticket), ph, pn, sh if H is not None else sn),
               self.home.handle)
