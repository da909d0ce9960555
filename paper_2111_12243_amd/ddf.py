"""ctypes binding of libddf (include/ddf.h) — argument marshalling only.

Every function keeps the C name.  Device buffers are passed as torch tensors (their
data_ptr()) or as integer device addresses; streams as torch.cuda.Stream, an integer
hipStream_t, or None for torch's current stream.  A non-OK status raises DDFError.  Every
step of the hot path runs in the library's kernels; this module computes nothing.  If the
library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddf.so")

DDF_SPMV, DDF_SPTRSV_LOWER = 0, 1
DDF_OP_SPMV, DDF_OP_SPMV_ADJ, DDF_OP_SPTRSV, DDF_OP_SPTRSV_ADJ, DDF_OP_SPTRSV_T = 0, 1, 2, 3, 4
DDF_OP_SPMV_ADJ_KERNEL, DDF_OP_SPTRSV_ADJ_KERNEL = 5, 6
STATUS = ["DDF_OK", "DDF_E_ARG", "DDF_E_CSR", "DDF_E_NOT_LOWER", "DDF_E_NO_DIAG", "DDF_E_KIND",
          "DDF_E_NOMEM", "DDF_E_HIP", "DDF_E_DEVICE", "DDF_E_UNSUPPORTED"]
(DDF_OK, DDF_E_ARG, DDF_E_CSR, DDF_E_NOT_LOWER, DDF_E_NO_DIAG, DDF_E_KIND, DDF_E_NOMEM, DDF_E_HIP,
 DDF_E_DEVICE, DDF_E_UNSUPPORTED) = range(10)

EXPORTED = [
    "ddf_sptrsv_adjoint_noalloc",
    "ddf_plan_time_kernels", "ddf_plan_kernel_time",
    "ddf_opts_default", "ddf_inspect", "ddf_inspect_batch", "ddf_plan_destroy", "ddf_spmv",
    "ddf_spmv_v", "ddf_sptrsv", "ddf_sptrsv_v", "ddf_spmv_adjoint", "ddf_sptrsv_adjoint", "ddf_sptrsv_value_grad",
    "ddf_sptrsv_batch", "ddf_sptrsv_batch_adjoint", "ddf_graph_create_batch", "ddf_graph_launch",
    "ddf_graph_destroy", "ddf_plain_spmv", "ddf_plain_sptrsv", "ddf_plain_spmv_adjoint",
    "ddf_plain_sptrsv_adjoint", "ddf_sptrsv_batch_per_matrix", "ddf_autotune", "ddf_plan_info",
    "ddf_plan_export", "ddf_plan_device_tables", "ddf_plan_traffic", "ddf_plan_sync_status", "ddf_plan_set_spin_limit",
    "ddf_status_string", "ddf_last_error", "ddf_version",
]


class DDFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS[status] if 0 <= status < len(STATUS) else status}: {msg}")
        self.status = status


class ddf_opts(C.Structure):
    _fields_ = [("window", C.c_int32), ("build_adjoint", C.c_int32), ("host_only", C.c_int32),
                ("threads", C.c_int32), ("ops_per_lane", C.c_int32), ("rows_passes", C.c_int32),
                ("xcd_remap", C.c_int32), ("solve_blocks", C.c_int32),
                ("solve_path", C.c_int32), ("thin_helpers", C.c_int32), ("thin_ahead", C.c_int32),
                ("thin_ring", C.c_int32), ("thin_lanes", C.c_int32), ("only_blas", C.c_int32)]


class ddf_csr_host(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p)]


class ddf_plan_tables_t(C.Structure):
    _fields_ = [("header", C.POINTER(C.c_int64)), ("part_ptr", C.POINTER(C.c_int64)),
                ("part_rows", C.POINTER(C.c_int64)), ("regions", C.POINTER(C.c_int64)),
                ("codelets", C.POINTER(C.c_int64)), ("aux", C.POINTER(C.c_int32)),
                ("perm", C.POINTER(C.c_int32))]


class ddf_device_tables_t(C.Structure):
    _fields_ = [("cods", C.POINTER(C.c_int32)), ("aux", C.POINTER(C.c_int32)), ("tasks", C.POINTER(C.c_int32)),
                ("sync", C.POINTER(C.c_int32)), ("tasksN", C.POINTER(C.c_int32)), ("n_cods", C.c_int64),
                ("aux_len", C.c_int64), ("n_tasks", C.c_int64), ("n_counters", C.c_int64), ("n_tasksN", C.c_int64),
                ("thin_rec", C.POINTER(C.c_int32)), ("thin_lvl", C.POINTER(C.c_int32)),
                ("thin_rows", C.POINTER(C.c_int32)), ("n_thin_rec", C.c_int64),
                ("n_thin_lvl", C.c_int64), ("thin_lg", C.c_int32), ("thin_ring_size", C.c_int32),
                ("thin_reserved", C.c_int32), ("thin_ngs", C.c_int32), ("thin_block", C.c_int32),
                ("reserved", C.c_int32), ("rowlist", C.POINTER(C.c_int32)), ("n_rowlist", C.c_int64),
                ("df_tasks", C.POINTER(C.c_int32)), ("n_df_tasks", C.c_int64), ("df_ptr", C.POINTER(C.c_int64)),
                ("n_df_ptr", C.c_int64), ("df_lcols", C.POINTER(C.c_int32)), ("n_df_lcols", C.c_int64),
                ("df_group", C.c_int32), ("df_reserved", C.c_int32), ("df_slots", C.POINTER(C.c_int32)),
                ("n_df_slots", C.c_int64)]


class ddf_plan_info_t(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nmat", C.c_int32), ("n_rows", C.c_int32), ("n_cols", C.c_int32),
                ("nnz", C.c_int64), ("n_parts", C.c_int64), ("n_regions", C.c_int64),
                ("n_codelets", C.c_int64), ("aux_len", C.c_int64), ("codelets_by_type", C.c_int64 * 3),
                ("ops_by_type", C.c_int64 * 3), ("n_tasks", C.c_int64), ("n_tasks_adjoint", C.c_int64),
                ("dev_plan_bytes", C.c_int64), ("dev_plan_bytes_adj", C.c_int64),
                ("has_adjoint", C.c_int32), ("max_levels", C.c_int32), ("inspect_seconds", C.c_double),
                ("hash", C.c_uint64), ("ops_per_lane", C.c_int32), ("rows_passes", C.c_int32),
                ("xcd_remap", C.c_int32), ("solve_path", C.c_int32), ("solve_path_adj", C.c_int32),
                ("reserved", C.c_int32), ("phase_seconds", C.c_double * 5)]


_LIB = None


def lib():
    """The loaded libddf.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "ddf_opts_default": (None, [C.POINTER(ddf_opts)]),
            "ddf_inspect": (I32, [I32, C.POINTER(ddf_csr_host), C.POINTER(ddf_opts), C.POINTER(P)]),
            "ddf_inspect_batch": (I32, [I32, I32, C.POINTER(ddf_csr_host), P, C.POINTER(ddf_opts), C.POINTER(P)]),
            "ddf_plan_destroy": (I32, [P]),
            "ddf_spmv": (I32, [P, P, P, I32, P]),
            "ddf_spmv_v": (I32, [P, P, P, P, I32, P]),
            "ddf_sptrsv": (I32, [P, P, P, I32, P]),
            "ddf_sptrsv_v": (I32, [P, P, P, P, I32, P]),
            "ddf_spmv_adjoint": (I32, [P, P, P, P, P, P, I32, P]),
            "ddf_sptrsv_adjoint": (I32, [P, P, P, P, P, P, I32, P]),
            "ddf_sptrsv_value_grad": (I32, [P, P, P, P, I32, P]),
            "ddf_sptrsv_adjoint_noalloc": (I32, [P, P, P, P, P, P, I32, P]),
            "ddf_sptrsv_batch": (I32, [P, P, P, P, P]),
            "ddf_sptrsv_batch_adjoint": (I32, [P, P, P, P, P, P, P]),
            "ddf_graph_create_batch": (I32, [P, I32, P, P, P, P, P, C.POINTER(P)]),
            "ddf_graph_launch": (I32, [P, P]),
            "ddf_graph_destroy": (I32, [P]),
            "ddf_plain_spmv": (I32, [P, P, P, P, I32, P]),
            "ddf_plain_sptrsv": (I32, [P, P, P, P, I32, P]),
            "ddf_plain_spmv_adjoint": (I32, [P, P, P, P, P, P, I32, P]),
            "ddf_plain_sptrsv_adjoint": (I32, [P, P, P, P, P, P, I32, P]),
            "ddf_sptrsv_batch_per_matrix": (I32, [P, P, P, P, P]),
            "ddf_autotune": (I32, [P, I32, I32, P, D]),
            "ddf_plan_info": (I32, [P, C.POINTER(ddf_plan_info_t)]),
            "ddf_plan_export": (I32, [P, I32, I32, C.POINTER(ddf_plan_tables_t)]),
            "ddf_plan_device_tables": (I32, [P, I32, C.POINTER(ddf_device_tables_t)]),
            "ddf_plan_traffic": (I32, [P, I32, I32, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
            "ddf_plan_sync_status": (I32, [P, P]),
            "ddf_plan_set_spin_limit": (I32, [P, I64]),
            "ddf_plan_time_kernels": (I32, [P, I32]),
            "ddf_plan_kernel_time": (I32, [P, C.POINTER(D), C.POINTER(I64), C.POINTER(I64)]),
            "ddf_status_string": (C.c_char_p, [I32]),
            "ddf_last_error": (C.c_char_p, []),
            "ddf_version": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(st):
    if st != DDF_OK:
        raise DDFError(st, lib().ddf_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    raise TypeError(f"cannot pass {type(a)} as a buffer")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Plan:
    """Owns a ddf_plan_t; destroyed with ddf_plan_destroy."""

    def __init__(self, handle, kind, shape, keep=()):
        self.handle = handle
        self.kind = kind
        self.n_rows, self.n_cols = shape
        self._keep = keep

    def close(self):
        if self.handle:
            lib().ddf_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return self.handle


def ddf_opts_default(**kw) -> ddf_opts:
    o = ddf_opts()
    lib().ddf_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, int(v))
    return o


def _host_csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    vals = getattr(A, "values", None)
    v = np.ascontiguousarray(vals, dtype=np.float64) if vals is not None else None
    h = ddf_csr_host(int(A.n_rows), int(A.n_cols), rp.ctypes.data, ci.ctypes.data,
                     v.ctypes.data if v is not None else None)
    return h, (rp, ci, v)


def ddf_inspect(kind, A, opts: ddf_opts | None = None) -> Plan:
    h, keep = _host_csr(A)
    out = C.c_void_p()
    _check(lib().ddf_inspect(kind, C.byref(h), C.byref(opts) if opts else None, C.byref(out)))
    return Plan(out.value, kind, (A.n_rows, A.n_cols))


def ddf_inspect_batch(kind, mats, nrhs, opts: ddf_opts | None = None) -> Plan:
    arr = (ddf_csr_host * len(mats))()
    keep = []
    for i, A in enumerate(mats):
        h, kp = _host_csr(A)
        arr[i] = h
        keep.append(kp)
    k = np.ascontiguousarray(nrhs, dtype=np.int32)
    out = C.c_void_p()
    _check(lib().ddf_inspect_batch(kind, len(mats), arr, k.ctypes.data,
                                   C.byref(opts) if opts else None, C.byref(out)))
    return Plan(out.value, kind, (sum(A.n_rows for A in mats), sum(A.n_cols for A in mats)))


def ddf_plan_destroy(plan: Plan):
    plan.close()


def ddf_spmv(plan, x, y, nrhs, stream=None):
    _check(lib().ddf_spmv(plan.handle, _ptr(x), _ptr(y), nrhs, _stream(stream)))


def ddf_spmv_v(plan, vals, x, y, nrhs, stream=None):
    _check(lib().ddf_spmv_v(plan.handle, _ptr(vals), _ptr(x), _ptr(y), nrhs, _stream(stream)))


def ddf_sptrsv(plan, b, x, nrhs, stream=None):
    _check(lib().ddf_sptrsv(plan.handle, _ptr(b), _ptr(x), nrhs, _stream(stream)))


def ddf_sptrsv_v(plan, vals, b, x, nrhs, stream=None):
    _check(lib().ddf_sptrsv_v(plan.handle, _ptr(vals), _ptr(b), _ptr(x), nrhs, _stream(stream)))


def ddf_spmv_adjoint(plan, vals, x, gy, gx, gvals, nrhs, stream=None):
    _check(lib().ddf_spmv_adjoint(plan.handle, _ptr(vals), _ptr(x), _ptr(gy), _ptr(gx), _ptr(gvals),
                                  nrhs, _stream(stream)))


def ddf_sptrsv_adjoint(plan, vals, x, gx, gb, gvals, nrhs, stream=None):
    _check(lib().ddf_sptrsv_adjoint(plan.handle, _ptr(vals), _ptr(x), _ptr(gx), _ptr(gb), _ptr(gvals),
                                    nrhs, _stream(stream)))


def ddf_sptrsv_adjoint_noalloc(plan, vals, x, gx, gb, gvals, nrhs, stream=None):
    """ddf_sptrsv_adjoint with its scratch in the library's static device array (no allocation)."""
    _check(lib().ddf_sptrsv_adjoint_noalloc(plan.handle, _ptr(vals), _ptr(x), _ptr(gx), _ptr(gb), _ptr(gvals),
                                            nrhs, _stream(stream)))


def ddf_sptrsv_value_grad(plan, x, gb, gvals, nrhs, stream=None):
    _check(lib().ddf_sptrsv_value_grad(plan.handle, _ptr(x), _ptr(gb), _ptr(gvals), nrhs, _stream(stream)))


def ddf_sptrsv_batch(plan, vals, b, x, stream=None):
    _check(lib().ddf_sptrsv_batch(plan.handle, _ptr(vals), _ptr(b), _ptr(x), _stream(stream)))


def ddf_sptrsv_batch_adjoint(plan, vals, x, gx, gb, gvals, stream=None):
    _check(lib().ddf_sptrsv_batch_adjoint(plan.handle, _ptr(vals), _ptr(x), _ptr(gx), _ptr(gb),
                                          _ptr(gvals), _stream(stream)))


def ddf_sptrsv_batch_per_matrix(plan, vals, b, x, stream=None):
    _check(lib().ddf_sptrsv_batch_per_matrix(plan.handle, _ptr(vals), _ptr(b), _ptr(x), _stream(stream)))


class Graph:
    def __init__(self, handle, keep=()):
        self.handle = handle
        self._keep = keep

    def close(self):
        if self.handle:
            lib().ddf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ddf_graph_create_batch(plan, adjoint, vals, inp, x, out, gvals) -> Graph:
    g = C.c_void_p()
    _check(lib().ddf_graph_create_batch(plan.handle, int(adjoint), _ptr(vals), _ptr(inp), _ptr(x), _ptr(out),
                                        _ptr(gvals), C.byref(g)))
    return Graph(g.value, (plan, vals, inp, x, out, gvals))


def ddf_graph_launch(graph, stream=None):
    _check(lib().ddf_graph_launch(graph.handle, _stream(stream)))


def ddf_graph_destroy(graph):
    graph.close()


def ddf_plain_spmv(plan, vals, x, y, nrhs, stream=None):
    _check(lib().ddf_plain_spmv(plan.handle, _ptr(vals), _ptr(x), _ptr(y), nrhs, _stream(stream)))


def ddf_plain_sptrsv(plan, vals, b, x, nrhs, stream=None):
    _check(lib().ddf_plain_sptrsv(plan.handle, _ptr(vals), _ptr(b), _ptr(x), nrhs, _stream(stream)))


def ddf_plain_spmv_adjoint(plan, vals, x, gy, gx, gvals, nrhs, stream=None):
    _check(lib().ddf_plain_spmv_adjoint(plan.handle, _ptr(vals), _ptr(x), _ptr(gy), _ptr(gx), _ptr(gvals),
                                        nrhs, _stream(stream)))


def ddf_plain_sptrsv_adjoint(plan, vals, x, gx, gb, gvals, nrhs, stream=None):
    _check(lib().ddf_plain_sptrsv_adjoint(plan.handle, _ptr(vals), _ptr(x), _ptr(gx), _ptr(gb), _ptr(gvals),
                                          nrhs, _stream(stream)))


def ddf_autotune(plan, op, nrhs, stream=None, budget_ms=0.0):
    _check(lib().ddf_autotune(plan.handle, op, nrhs, _stream(stream), float(budget_ms)))


def ddf_plan_info(plan) -> dict:
    o = ddf_plan_info_t()
    _check(lib().ddf_plan_info(plan.handle, C.byref(o)))
    d = {}
    for name, _ in ddf_plan_info_t._fields_:
        v = getattr(o, name)
        d[name] = list(v) if hasattr(v, "__len__") else v
    return d


def ddf_plan_export(plan, which=0, mat=0) -> dict:
    """Copies of the canonical tables (same layout as the oracle's)."""
    t = ddf_plan_tables_t()
    _check(lib().ddf_plan_export(plan.handle, which, mat, C.byref(t)))
    h = np.ctypeslib.as_array(t.header, shape=(9,)).copy()
    n_rows, npart, nreg, ncod, naux = int(h[1]), int(h[5]), int(h[6]), int(h[7]), int(h[8])

    def grab(p, n, dt):
        if n == 0 or not p:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(p, shape=(n,)).astype(dt, copy=True)

    out = {"header": h, "part_ptr": grab(t.part_ptr, npart + 1, np.int64),
           "part_rows": grab(t.part_rows, n_rows, np.int64),
           "regions": grab(t.regions, nreg * 8, np.int64).reshape(nreg, 8),
           "codelets": grab(t.codelets, ncod * 18, np.int64).reshape(ncod, 18),
           "aux": grab(t.aux, naux, np.int32)}
    if which == 1:
        out["perm"] = grab(t.perm, int(h[3]), np.int64)
    return out


def ddf_plan_device_tables(plan, which=0) -> dict:
    """Copies of the tables the kernels read (records, aux, tasks, groups, level bounds)."""
    t = ddf_device_tables_t()
    _check(lib().ddf_plan_device_tables(plan.handle, which, C.byref(t)))

    def grab(p, n, cols=None):
        if n == 0 or not p:
            a = np.zeros(0, dtype=np.int32)
        else:
            a = np.ctypeslib.as_array(p, shape=(n * (cols or 1),)).copy()
        return a.reshape(-1, cols) if cols else a

    sync = grab(t.sync, t.n_tasks, 4) if t.sync else np.zeros((0, 4), np.int32)
    return {"cods": grab(t.cods, t.n_cods, 16), "aux": grab(t.aux, t.aux_len), "tasks": grab(t.tasks, t.n_tasks, 4),
            "sync": sync, "n_counters": int(t.n_counters), "tasksN": grab(t.tasksN, t.n_tasksN, 4),
            "thin_rec": grab(t.thin_rec, t.n_thin_rec, 21), "thin_lvl": grab(t.thin_lvl, t.n_thin_lvl, 4),
            "thin_rows": grab(t.thin_rows, t.n_thin_lvl and ddf_plan_info(plan)["n_rows"], 1).ravel(),
            "thin_lg": int(t.thin_lg), "thin_ring_size": int(t.thin_ring_size), "thin_ngs": int(t.thin_ngs),
            "thin_block": int(t.thin_block), "rowlist": grab(t.rowlist, t.n_rowlist),
            "df_tasks": grab(t.df_tasks, t.n_df_tasks, 4), "df_lcols": grab(t.df_lcols, t.n_df_lcols), "df_group": int(t.df_group), "df_slots": grab(t.df_slots, t.n_df_slots, 2),
            "df_ptr": (np.ctypeslib.as_array(t.df_ptr, shape=(t.n_df_ptr,)).copy() if t.n_df_ptr
                       else np.zeros(0, np.int64))}


def ddf_plan_time_kernels(plan, enable=1) -> None:
    """Start (1) or stop (0) timing the main kernel of each execution call on the plan."""
    _check(lib().ddf_plan_time_kernels(plan.handle, int(enable)))


def ddf_plan_kernel_time(plan) -> tuple:
    """(total ms, timed calls, kernel launches) of the calls timed since ddf_plan_time_kernels."""
    ms, calls, launches = C.c_double(), C.c_int64(), C.c_int64()
    _check(lib().ddf_plan_kernel_time(plan.handle, C.byref(ms), C.byref(calls), C.byref(launches)))
    return ms.value, calls.value, launches.value


def ddf_plan_traffic(plan, op, nrhs) -> tuple:
    """(algorithmic bytes, CSR-equivalent bytes, flops) of one call."""
    a, b, f = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().ddf_plan_traffic(plan.handle, op, nrhs, C.byref(a), C.byref(b), C.byref(f)))
    return a.value, b.value, f.value


def ddf_plan_sync_status(plan, stream=None):
    _check(lib().ddf_plan_sync_status(plan.handle, _stream(stream)))


def ddf_plan_set_spin_limit(plan, limit):
    _check(lib().ddf_plan_set_spin_limit(plan.handle, int(limit)))


def ddf_status_string(s) -> str:
    return lib().ddf_status_string(int(s)).decode()


def ddf_last_error() -> str:
    return lib().ddf_last_error().decode()


def ddf_version() -> str:
    return lib().ddf_version().decode()
