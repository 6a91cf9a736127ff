"""ctypes binding of libpfc.so (declared in include/pfc.h).

Argument marshalling only: every function forwards to the C entry point of
the same name.  Device arrays are torch tensors on the current HIP device
(float64, contiguous); host arrays are numpy arrays.  torch supplies device
memory and the current stream, nothing else.  If the library has not been
built, importing this module raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PFC_LIBRARY selects another build of the library (the instrumented one of phase_probe.py)
LIB_PATH = os.environ.get("PFC_LIBRARY") or os.path.join(_HERE, "libpfc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1501_06852_amd.build` (or __graft_entry__.build())")

# torch first: its ROCm build carries its own HIP runtime, which must be the one
# loaded in the process before this library binds to libamdhip64 (the other
# order leaves torch's runtime without a device)
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# status codes (pfc.h)
PFC_OK = 0
PFC_NOT_CONVERGED = 1
PFC_WARN_TAU_CRITICAL = 2
PFC_ERR_ARG = -1
PFC_ERR_OOM = -2
PFC_ERR_HIP = -3
PFC_ERR_BREAKDOWN = -4
PFC_ERR_ADMISSION = -5
PFC_ERR_STATE = -6
PFC_FP64 = 0
PFC_MIXED = 1
PFC_INIT_GIVEN = 0
PFC_INIT_CONSISTENT = 1
PFC_OP_M = 0
PFC_OP_K = 1
PFC_MODEL_PFC2 = 0
PFC_MODEL_PFC1 = 1
PFC_GAMMA_SCALE_ROW = 0
PFC_GAMMA_LITERAL = 1


class pfc_opts(C.Structure):
    _fields_ = [("struct_size", C.c_int), ("precision", C.c_int), ("restart", C.c_int), ("max_steps", C.c_int),
                ("outer_tol", C.c_double), ("inner_tol", C.c_double), ("inner_maxit", C.c_int),
                ("shared_ops", C.c_int), ("rows_per_thread", C.c_int), ("max_run_steps", C.c_int),
                ("ticks_per_graph", C.c_int), ("single_reduction", C.c_int),
                ("schur_variant", C.c_int), ("sd_iters", C.c_int), ("model", C.c_int), ("psi_min", C.c_double),
                ("grid_columns", C.c_int), ("gamma_mode", C.c_int), ("inner_fixed", C.c_int * 5),
                ("pcg_steps_per_launch", C.c_int)]


class pfc_solve_info(C.Structure):
    _fields_ = [("status", C.c_int), ("outer_iters", C.c_int), ("cycles", C.c_int), ("inner_applies", C.c_int),
                ("inner_total", C.c_longlong), ("inner_max", C.c_int * 5), ("reserved", C.c_int),
                ("est_rel_res", C.c_double), ("true_rel_res", C.c_double), ("t_solve", C.c_double)]

    def as_dict(self):
        return dict(status=self.status, outer_iters=self.outer_iters, cycles=self.cycles,
                    inner_applies=self.inner_applies, inner_total=int(self.inner_total),
                    inner_max=list(self.inner_max), est_rel_res=self.est_rel_res, true_rel_res=self.true_rel_res,
                    t_solve=self.t_solve)


class pfc_schedule(C.Structure):
    _fields_ = [("n_cycles", C.c_int), ("cycle_len", C.POINTER(C.c_int)), ("n_applies", C.c_int),
                ("inner_counts", C.POINTER(C.c_int))]


class pfc_server_opts(C.Structure):
    _fields_ = [("struct_size", C.c_int), ("precision", C.c_int), ("hbm_budget", C.c_size_t),
                ("max_slots", C.c_int), ("ticks_per_graph", C.c_int), ("rows_per_thread", C.c_int),
                ("tuned", C.c_int)]


class pfc_tune_entry(C.Structure):
    _fields_ = [("struct_size", C.c_int), ("arch", C.c_char * 32), ("dim", C.c_int), ("n", C.c_int), ("z", C.c_int),
                ("precision", C.c_int), ("count", C.c_int), ("rows_per_thread", C.c_int),
                ("ticks_per_graph", C.c_int), ("pcg_steps_per_launch", C.c_int), ("grid_columns", C.c_int),
                ("shared_ops", C.c_int), ("ms_per_step", C.c_double), ("ms_default", C.c_double),
                ("candidates", C.c_int), ("from_cache", C.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}
        d["arch"] = self.arch.decode()
        return d


class pfc_result(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("status", C.c_int), ("n_stages", C.c_int), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("state", C.POINTER(C.c_double)),
                ("infos", C.POINTER(pfc_solve_info))]


_vp = C.c_void_p
_ip = C.POINTER(C.c_int)
_dp = C.POINTER(C.c_double)


def _sig(name, res, args):
    f = getattr(_lib, name, None)
    if f is None:
        return None
    f.restype = res
    f.argtypes = args
    return f


_sig("pfc_status_str", C.c_char_p, [C.c_int])
_sig("pfc_last_error", C.c_char_p, [])
_sig("pfc_opts_default", None, [C.POINTER(pfc_opts)])
_sig("pfc_tau_critical", C.c_double, [C.c_double, C.c_double])
_sig("pfc_mesh_create_p1", C.c_int, [C.c_int, C.c_int, C.c_int, _ip, _dp, C.POINTER(_vp)])
_sig("pfc_mesh_create_p2", C.c_int, [C.c_int, C.c_int, C.c_int, _ip, _dp, C.POINTER(_vp)])
_sig("pfc_mesh_create_csr", C.c_int, [C.c_int, C.c_int, C.c_int, _ip, _ip, _dp, _dp, C.c_int, _ip, _dp, C.POINTER(_vp)])
_sig("pfc_mesh_create_csr_device", C.c_int, [C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp, C.c_int, _vp, _vp,
                                              C.POINTER(_vp)])
_sig("pfc_mesh_query", C.c_int, [_vp, _ip, _ip, _ip, _ip])
_sig("pfc_mesh_grid_side", C.c_int, [_vp, _ip])
_sig("pfc_mesh_export_csr", C.c_int, [_vp, _ip, _ip, _dp, _dp])
_sig("pfc_mesh_destroy", None, [_vp])
_sig("pfc_spmv", C.c_int, [_vp, C.c_int, _vp, _vp, _vp])
_sig("pfc_assemble_N", C.c_int, [_vp, _vp, _vp, _vp])
_sig("pfc_load_psi3", C.c_int, [_vp, _vp, _vp, _vp])
_sig("pfc_instance_footprint", C.c_size_t, [_vp, C.POINTER(pfc_opts)])
_sig("pfc_instance_create", C.c_int, [_vp, C.POINTER(pfc_opts), C.POINTER(_vp)])
_sig("pfc_instance_destroy", None, [_vp])
_sig("pfc_solve", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, _vp, _vp,
                            C.POINTER(pfc_schedule), C.POINTER(pfc_solve_info), _vp])
_sig("pfc_solve_x", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, _vp, _vp,
                              C.POINTER(pfc_schedule), C.POINTER(pfc_solve_info), _vp])
_sig("pfc_last_inner_counts", C.c_int, [_vp, _ip, C.c_int, _ip])
_sig("pfc_instance_launch_stats", C.c_int, [_vp, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)])
_sig("pfc_instance_config", C.c_int, [_vp, _ip, _ip, _ip, _ip])
_sig("pfc_rosenbrock_run", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                     C.POINTER(pfc_schedule), C.POINTER(pfc_solve_info), _vp])
_sig("pfc_rosenbrock_adaptive", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_int, C.c_int, _dp, _ip, _ip, C.POINTER(pfc_solve_info),
                                          _vp])
_sig("pfc_apply_AR", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, _vp, _vp, _vp])
_sig("pfc_apply_AR_x", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, _vp, _vp, _vp])
_sig("pfc_apply_AR_noalloc", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, _vp, _vp, _vp])
_sig("pfc_apply_pch", C.c_int, [_vp, C.c_double, _vp, _vp, _ip, _ip, _vp])
_sig("pfc_stage_rhs", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, C.c_double, _vp, _vp])
_sig("pfc_batch_run", C.c_int, [C.POINTER(_vp), C.c_int, C.POINTER(_vp), _dp, _dp, _dp, C.c_int, C.c_int,
                                C.POINTER(pfc_solve_info), _vp])
_sig("pfc_autotune", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.POINTER(pfc_tune_entry), _vp])
_sig("pfc_autotune_mix", C.c_int, [C.POINTER(_vp), C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(pfc_tune_entry), _vp])
_sig("pfc_tune_lookup", C.c_int, [C.c_char_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(pfc_tune_entry)])
_sig("pfc_tune_load", C.c_int, [C.c_char_p])
_sig("pfc_tune_save", C.c_int, [C.c_char_p])
_sig("pfc_tune_clear", None, [])
_sig("pfc_server_create", C.c_int, [C.POINTER(pfc_server_opts), C.POINTER(_vp)])
_sig("pfc_server_submit", C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double, _dp, C.c_int, C.c_uint64])
_sig("pfc_server_poll", C.c_int, [_vp, C.POINTER(pfc_result), C.c_int, _ip])
_sig("pfc_result_free", None, [C.POINTER(pfc_result)])
_sig("pfc_server_drain", C.c_int, [_vp])
_sig("pfc_server_clock", C.c_double, [_vp])
_sig("pfc_server_destroy", None, [_vp])

# every symbol declared in include/pfc.h
DECLARED = [
    "pfc_status_str", "pfc_last_error", "pfc_opts_default", "pfc_tau_critical", "pfc_mesh_create_p1", "pfc_mesh_create_p2",
    "pfc_mesh_create_csr", "pfc_mesh_create_csr_device", "pfc_mesh_query", "pfc_mesh_grid_side", "pfc_mesh_export_csr", "pfc_mesh_destroy", "pfc_spmv",
    "pfc_assemble_N", "pfc_load_psi3", "pfc_instance_footprint", "pfc_instance_create", "pfc_instance_destroy",
    "pfc_solve", "pfc_solve_x", "pfc_last_inner_counts", "pfc_instance_launch_stats", "pfc_instance_config",
    "pfc_rosenbrock_run",
    "pfc_rosenbrock_adaptive", "pfc_apply_AR", "pfc_apply_AR_x", "pfc_apply_AR_noalloc", "pfc_apply_pch", "pfc_stage_rhs",
    "pfc_batch_run", "pfc_autotune", "pfc_autotune_mix", "pfc_tune_lookup", "pfc_tune_load", "pfc_tune_save", "pfc_tune_clear",
    "pfc_server_create", "pfc_server_submit", "pfc_server_poll", "pfc_result_free",
    "pfc_server_drain", "pfc_server_clock", "pfc_server_destroy",
]


class PFCError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.pfc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.pfc_status_str(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code, where):
    if code < 0:
        raise PFCError(code, where)
    return code


def pfc_status_str(code: int) -> str:
    return _lib.pfc_status_str(code).decode()


def pfc_last_error() -> str:
    return _lib.pfc_last_error().decode()


def pfc_tau_critical(r: float, psibar: float) -> float:
    return _lib.pfc_tau_critical(r, psibar)


def pfc_opts_default(**over) -> pfc_opts:
    o = pfc_opts()
    _lib.pfc_opts_default(C.byref(o))
    for k, v in over.items():
        if k == "inner_fixed":
            v = (C.c_int * 5)(*v)
        setattr(o, k, v)
    return o


# ---- helpers for array arguments -------------------------------------------------
def _host_i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _host_f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _dev(t, numel=None, name="tensor"):
    """Device pointer of a contiguous float64 torch tensor on the GPU."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return _vp(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _sched(s):
    """(cycles, inner_counts) -> pfc_schedule with owned buffers."""
    cyc, inn = s
    cyc = np.ascontiguousarray(cyc, dtype=np.int32)
    inn = np.ascontiguousarray(np.asarray(inn, dtype=np.int32).reshape(-1))
    q = pfc_schedule(len(cyc), cyc.ctypes.data_as(_ip), len(inn) // 5, inn.ctypes.data_as(_ip))
    return q, (cyc, inn)


# ---- meshes ------------------------------------------------------------------------
def pfc_mesh_create_p1(dim, n, elem_nodes, elem_coords):
    en, pen = _host_i32(elem_nodes)
    ec, pec = _host_f64(elem_coords)
    if en.size % (dim + 1) or ec.size != en.size * dim:
        raise ValueError("elem_nodes / elem_coords shapes do not match dim")
    h = _vp()
    _check(_lib.pfc_mesh_create_p1(dim, n, en.size // (dim + 1), pen, pec, C.byref(h)), "pfc_mesh_create_p1")
    return h


def pfc_mesh_create_p2(dim, n, elem_nodes, elem_coords):
    """elem_nodes [n_elem, (dim+1)(dim+2)/2] (vertices, then edges), elem_coords [n_elem, dim+1, dim]."""
    en, pen = _host_i32(elem_nodes)
    ec, pec = _host_f64(elem_coords)
    q = (dim + 1) * (dim + 2) // 2
    if en.size % q or ec.size != (en.size // q) * (dim + 1) * dim:
        raise ValueError("elem_nodes / elem_coords shapes do not match dim")
    h = _vp()
    _check(_lib.pfc_mesh_create_p2(dim, n, en.size // q, pen, pec, C.byref(h)), "pfc_mesh_create_p2")
    return h


def pfc_mesh_create_csr(dim, n, row_ptr, col_idx, M_val, K_val, elem_nodes, elem_vol):
    rp, prp = _host_i32(row_ptr)
    ci, pci = _host_i32(col_idx)
    mv, pmv = _host_f64(M_val)
    kv, pkv = _host_f64(K_val)
    en, pen = _host_i32(elem_nodes)
    ev, pev = _host_f64(elem_vol)
    h = _vp()
    _check(_lib.pfc_mesh_create_csr(dim, n, ci.size, prp, pci, pmv, pkv, ev.size, pen, pev, C.byref(h)),
           "pfc_mesh_create_csr")
    return h


def _dev_any(t, dtype, name):
    """Device pointer of a contiguous torch tensor of `dtype` on the GPU."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    return _vp(t.data_ptr())


def pfc_mesh_create_csr_device(dim, n, row_ptr, col_idx, M_val, K_val, elem_nodes, elem_vol):
    """As pfc_mesh_create_csr with every array a torch tensor on the GPU (int32 indices, float64 values)."""
    import torch
    args = [_dev_any(row_ptr, torch.int32, "row_ptr"), _dev_any(col_idx, torch.int32, "col_idx"),
            _dev_any(M_val, torch.float64, "M_val"), _dev_any(K_val, torch.float64, "K_val")]
    en, ev = _dev_any(elem_nodes, torch.int32, "elem_nodes"), _dev_any(elem_vol, torch.float64, "elem_vol")
    h = _vp()
    _check(_lib.pfc_mesh_create_csr_device(dim, n, col_idx.numel(), *args, elem_vol.numel(), en, ev, C.byref(h)),
           "pfc_mesh_create_csr_device")
    return h


def pfc_mesh_query(mesh):
    d, n, z, e = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    _check(_lib.pfc_mesh_query(mesh, C.byref(d), C.byref(n), C.byref(z), C.byref(e)), "pfc_mesh_query")
    return dict(dim=d.value, n=n.value, nnz=z.value, n_elem=e.value)


def pfc_mesh_grid_side(mesh) -> int:
    N = C.c_int()
    _check(_lib.pfc_mesh_grid_side(mesh, C.byref(N)), "pfc_mesh_grid_side")
    return N.value


def pfc_mesh_export_csr(mesh):
    q = pfc_mesh_query(mesh)
    rp = np.empty(q["n"] + 1, np.int32)
    ci = np.empty(q["nnz"], np.int32)
    mv = np.empty(q["nnz"])
    kv = np.empty(q["nnz"])
    _check(_lib.pfc_mesh_export_csr(mesh, rp.ctypes.data_as(_ip), ci.ctypes.data_as(_ip), mv.ctypes.data_as(_dp),
                                    kv.ctypes.data_as(_dp)), "pfc_mesh_export_csr")
    return rp, ci, mv, kv


def pfc_mesh_destroy(mesh):
    _lib.pfc_mesh_destroy(mesh)


def pfc_spmv(mesh, which, x, y, stream=None):
    n = pfc_mesh_query(mesh)["n"]
    return _check(_lib.pfc_spmv(mesh, which, _dev(x, n, "x"), _dev(y, n, "y"), _stream(stream)), "pfc_spmv")


def pfc_assemble_N(mesh, psi, N_csr, stream=None):
    q = pfc_mesh_query(mesh)
    return _check(_lib.pfc_assemble_N(mesh, _dev(psi, q["n"], "psi"), _dev(N_csr, q["nnz"], "N_csr"),
                                      _stream(stream)), "pfc_assemble_N")


def pfc_load_psi3(mesh, psi, g, stream=None):
    n = pfc_mesh_query(mesh)["n"]
    return _check(_lib.pfc_load_psi3(mesh, _dev(psi, n, "psi"), _dev(g, n, "g"), _stream(stream)), "pfc_load_psi3")


# ---- instances ----------------------------------------------------------------------
def pfc_instance_footprint(mesh, opts):
    return _lib.pfc_instance_footprint(mesh, C.byref(opts))


def pfc_instance_create(mesh, opts):
    h = _vp()
    _check(_lib.pfc_instance_create(mesh, C.byref(opts), C.byref(h)), "pfc_instance_create")
    return h


def pfc_instance_destroy(inst):
    _lib.pfc_instance_destroy(inst)


def pfc_solve(inst, n, psi_k, r, psibar, tau, m11, rhs, x, replay=None, stream=None):
    """Returns (status, info dict).  replay: None or (cycle_lengths, inner_counts[apply][5])."""
    info = pfc_solve_info()
    keep = None
    rp = None
    if replay is not None:
        q, keep = _sched(replay)
        rp = C.byref(q)
    st = _lib.pfc_solve(inst, _dev(psi_k, n, "psi_k"), r, psibar, tau, m11, _dev(rhs, 3 * n, "rhs"),
                        _dev(x, 3 * n, "x"), rp, C.byref(info), _stream(stream))
    _check(st, "pfc_solve")
    del keep
    return st, info.as_dict()


def pfc_solve_x(inst, n, x_k, r, psibar, tau, m11, rhs, x, replay=None, stream=None):
    """pfc_solve at the full state x_k [3n] (required for PFC1 instances).  Returns (status, info dict)."""
    info = pfc_solve_info()
    keep = None
    rp = None
    if replay is not None:
        q, keep = _sched(replay)
        rp = C.byref(q)
    st = _lib.pfc_solve_x(inst, _dev(x_k, 3 * n, "x_k"), r, psibar, tau, m11, _dev(rhs, 3 * n, "rhs"),
                          _dev(x, 3 * n, "x"), rp, C.byref(info), _stream(stream))
    _check(st, "pfc_solve_x")
    del keep
    return st, info.as_dict()


def pfc_last_inner_counts(inst, cap=1000):
    buf = np.zeros((cap, 5), np.int32)
    na = C.c_int()
    _check(_lib.pfc_last_inner_counts(inst, buf.ctypes.data_as(_ip), cap, C.byref(na)), "pfc_last_inner_counts")
    return buf[:min(na.value, cap)].copy()


def pfc_instance_launch_stats(inst):
    a, b = C.c_longlong(), C.c_longlong()
    _check(_lib.pfc_instance_launch_stats(inst, C.byref(a), C.byref(b)), "pfc_instance_launch_stats")
    return a.value, b.value


def pfc_autotune(mesh, precision, count, force=False, stream=None):
    """Tune (or take from the table) the launch configuration of `count` instances; returns a dict."""
    e = pfc_tune_entry()
    e.struct_size = C.sizeof(pfc_tune_entry)
    _check(_lib.pfc_autotune(mesh, precision, count, 1 if force else 0, C.byref(e), _stream(stream)), "pfc_autotune")
    return e.as_dict()


def pfc_autotune_mix(meshes, precision, count, force=False, stream=None):
    """Tune the rows per thread of batches mixing the given meshes (the server's table entry); returns a dict."""
    e = pfc_tune_entry()
    e.struct_size = C.sizeof(pfc_tune_entry)
    arr = (_vp * len(meshes))(*[m.value if isinstance(m, _vp) else m for m in meshes])
    _check(_lib.pfc_autotune_mix(arr, len(meshes), precision, count, 1 if force else 0, C.byref(e), _stream(stream)),
           "pfc_autotune_mix")
    return e.as_dict()


def pfc_tune_lookup(dim, n, z, precision, count, arch=None):
    """The table's entry (dict) for `count` instances, or None."""
    e = pfc_tune_entry()
    rc = _lib.pfc_tune_lookup(None if arch is None else arch.encode(), dim, n, z, precision, count, C.byref(e))
    if rc == PFC_ERR_STATE:
        return None
    _check(rc, "pfc_tune_lookup")
    return e.as_dict()


def pfc_tune_load(path):
    return _check(_lib.pfc_tune_load(os.fsencode(path)), "pfc_tune_load")


def pfc_tune_save(path):
    return _check(_lib.pfc_tune_save(os.fsencode(path)), "pfc_tune_save")


def pfc_tune_clear():
    _lib.pfc_tune_clear()


def tuned_opts(entry, **kw):
    """pfc_opts for an instance of a tuned batch: the entry's choice plus explicit overrides."""
    base = dict(rows_per_thread=entry["rows_per_thread"], ticks_per_graph=entry["ticks_per_graph"],
                pcg_steps_per_launch=entry["pcg_steps_per_launch"], grid_columns=entry["grid_columns"],
                shared_ops=entry["shared_ops"])
    base.update(kw)
    return pfc_opts_default(**base)


def pfc_instance_config(inst):
    """The launch configuration of an instance served alone (dict)."""
    v = [C.c_int() for _ in range(4)]
    _check(_lib.pfc_instance_config(inst, *[C.byref(x) for x in v]), "pfc_instance_config")
    return dict(team_size=v[0].value, rows_per_thread=v[1].value, pcg_steps_per_launch=v[2].value,
                grid_columns=v[3].value)


def pfc_rosenbrock_run(inst, n, state, r, psibar, tau, n_steps, init=PFC_INIT_CONSISTENT, replays=None, stream=None):
    """Returns (status, list of per-stage info dicts)."""
    infos = (pfc_solve_info * max(1, 3 * n_steps))()
    rp = None
    keep = []
    if replays is not None:
        if len(replays) != 3 * n_steps:
            raise ValueError("need one schedule per stage solve")
        arr = (pfc_schedule * len(replays))()
        for k, s in enumerate(replays):
            q, kb = _sched(s)
            arr[k] = q
            keep.append(kb)
        rp = arr
    st = _lib.pfc_rosenbrock_run(inst, _dev(state, 3 * n, "state"), r, psibar, tau, n_steps, init, rp, infos,
                                 _stream(stream))
    _check(st, "pfc_rosenbrock_run")
    return st, [infos[k].as_dict() for k in range(3 * n_steps)]


def pfc_rosenbrock_adaptive(inst, n, state, r, psibar, tau0, t_end, rtol, atol, max_attempts=1000,
                            init=PFC_INIT_CONSISTENT, stream=None):
    """Returns (status, accepted taus, n_rejected, infos of the 3 stage solves of every attempted step)."""
    taus = np.zeros(max_attempts)
    na, nr = C.c_int(), C.c_int()
    infos = (pfc_solve_info * (3 * max_attempts))()
    st = _lib.pfc_rosenbrock_adaptive(inst, _dev(state, 3 * n, "state"), r, psibar, tau0, t_end, rtol, atol,
                                      max_attempts, init, taus.ctypes.data_as(_dp), C.byref(na), C.byref(nr),
                                      infos, _stream(stream))
    _check(st, "pfc_rosenbrock_adaptive")
    att = na.value + nr.value
    return st, taus[:na.value].copy(), nr.value, [infos[k].as_dict() for k in range(3 * att)]


def pfc_apply_AR(inst, n, psi_k, r, tau, m11, y, out, stream=None):
    return _check(_lib.pfc_apply_AR(inst, _dev(psi_k, n, "psi_k"), r, tau, m11, _dev(y, 3 * n, "y"),
                                    _dev(out, 3 * n, "out"), _stream(stream)), "pfc_apply_AR")


def pfc_apply_AR_x(inst, n, x_k, r, tau, m11, y, out, stream=None):
    return _check(_lib.pfc_apply_AR_x(inst, _dev(x_k, 3 * n, "x_k"), r, tau, m11, _dev(y, 3 * n, "y"),
                                      _dev(out, 3 * n, "out"), _stream(stream)), "pfc_apply_AR_x")


def pfc_apply_AR_noalloc(mesh, n, psi_k, r, tau, m11, y, out, stream=None):
    """Enqueues only (the C call returns without waiting); synchronise before reading `out`."""
    return _check(_lib.pfc_apply_AR_noalloc(mesh, _dev(psi_k, n, "psi_k"), r, tau, m11, _dev(y, 3 * n, "y"),
                                            _dev(out, 3 * n, "out"), _stream(stream)), "pfc_apply_AR_noalloc")


def pfc_apply_pch(inst, n, tau_s, v, z, fixed_counts=None, stream=None):
    cnt = np.zeros(5, np.int32)
    fc = None
    if fixed_counts is not None:
        fca = np.ascontiguousarray(fixed_counts, dtype=np.int32)
        fc = fca.ctypes.data_as(_ip)
    _check(_lib.pfc_apply_pch(inst, tau_s, _dev(v, 3 * n, "v"), _dev(z, 3 * n, "z"), fc, cnt.ctypes.data_as(_ip),
                              _stream(stream)), "pfc_apply_pch")
    return cnt


def pfc_stage_rhs(inst, n, x_k, ys, stage, r, tau, b, stream=None):
    return _check(_lib.pfc_stage_rhs(inst, _dev(x_k, 3 * n, "x_k"), _dev(ys, 9 * n, "ys"), stage, r, tau,
                                     _dev(b, 3 * n, "b"), _stream(stream)), "pfc_stage_rhs")


def pfc_batch_run(insts, ns, states, r, psibar, tau, n_steps, init=PFC_INIT_CONSISTENT, stream=None):
    """Returns (status, infos[count][3*n_steps] of dicts)."""
    cnt = len(insts)
    ih = (_vp * cnt)(*[i.value if isinstance(i, _vp) else i for i in insts])
    sp = (_vp * cnt)(*[_dev(s, 3 * n, "state").value for s, n in zip(states, ns)])
    ra, pr = _host_f64(r)
    pa, pp = _host_f64(psibar)
    ta, pt = _host_f64(tau)
    infos = (pfc_solve_info * max(1, cnt * 3 * n_steps))()
    st = _lib.pfc_batch_run(ih, cnt, sp, pr, pp, pt, n_steps, init, infos, _stream(stream))
    _check(st, "pfc_batch_run")
    out = [[infos[i * 3 * n_steps + k].as_dict() for k in range(3 * n_steps)] for i in range(cnt)]
    return st, out
