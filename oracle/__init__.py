"""CPU oracle for the DDF hot path — TEST INFRASTRUCTURE ONLY.

Plain FP64 loops in C (``ddf_oracle.c``, built with gcc -O2 -ffp-contract=off) wrapped with
ctypes.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the library never does, and this package never imports the library.

Every value function is the plain definition of its operation (row-by-row CSR products,
forward/backward substitution, their adjoints).  ``inspect`` is the paper's Algorithm 1
(Sec. IV-A) run step by step and returns the canonical plan tables:

    header   int64[9]  kind, n_rows, n_cols, nnz, t, n_parts, n_regions, n_codelets, aux_len
    part_ptr int64[n_parts+1], part_rows int64[n_rows]
    regions  int64[n_regions, 8]   part, pos0, T, first_codelet, chosen_strategy, cost[3]
    codelets int64[n_codelets, 18] type, flags, part, region, u, m, nn, P, row0, row_step,
                                   op0, op_step, col0, sigma0, sigma1, aux_off, aux_len, cost
    aux      int32[aux_len]
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

F_S0, F_S1, F_S2, F_SEP, F_RECT, F_RUNS = 1, 2, 4, 8, 16, 32
COD_FIELDS = ["type", "flags", "part", "region", "u", "m", "nn", "P", "row0", "row_step", "op0",
              "op_step", "col0", "sigma0", "sigma1", "aux_off", "aux_len", "cost"]
REG_FIELDS = ["part", "pos0", "T", "first_codelet", "chosen", "cost0", "cost1", "cost2"]


class _Plan(C.Structure):
    _fields_ = [("header", C.c_int64 * 9), ("part_ptr", C.POINTER(C.c_int64)),
                ("part_rows", C.POINTER(C.c_int64)), ("regions", C.POINTER(C.c_int64)),
                ("codelets", C.POINTER(C.c_int64)), ("aux", C.POINTER(C.c_int32))]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.orc_spmv.argtypes = [I32, P, P, P, I32, P, P]
        L.orc_sptrsv.argtypes = [I32, P, P, P, I32, P, P]
        L.orc_spmv_adj.argtypes = [I32, I32, P, P, P, I32, P, P, P, P]
        L.orc_sptrsv_adj.argtypes = [I32, P, P, P, I32, P, P, P, P, P]
        L.orc_levels.argtypes = [I32, P, P, P]
        L.orc_levels.restype = I64
        L.orc_validate.argtypes = [I32, I32, I32, P, P]
        L.orc_validate.restype = I32
        L.orc_transpose.argtypes = [I32, I32, P, P, P, P, P, P, P]
        L.orc_inspect.argtypes = [I32, I32, I32, P, P, I32, I32]
        L.orc_inspect.restype = C.POINTER(_Plan)
        L.orc_inspect_ex.argtypes = [I32, I32, I32, P, P, I32, I32, I32]
        L.orc_inspect_ex.restype = C.POINTER(_Plan)
        L.orc_plan_free.argtypes = [C.POINTER(_Plan)]
        L.orc_classify.argtypes = [I32, P, P, P, I64, P]
        L.orc_classify.restype = I32
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _csr(a):
    return (np.ascontiguousarray(a.row_ptr, dtype=np.int32),
            np.ascontiguousarray(a.col_idx, dtype=np.int32),
            np.ascontiguousarray(a.values, dtype=np.float64))


def _mat(X, n, k):
    X = np.ascontiguousarray(X, dtype=np.float64)
    return X.reshape(n, k)


def spmv(A, X):
    """Y = A X, X (n_cols, k)."""
    rp, ci, v = _csr(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    k = X.shape[1] if X.ndim == 2 else 1
    Y = np.empty((A.n_rows, k))
    lib().orc_spmv(A.n_rows, _p(rp), _p(ci), _p(v), k, _p(X), _p(Y))
    return Y


def sptrsv(L, B):
    """X with L X = B (L lower, diagonal last in each row)."""
    rp, ci, v = _csr(L)
    B = np.ascontiguousarray(B, dtype=np.float64)
    k = B.shape[1] if B.ndim == 2 else 1
    X = np.empty((L.n_rows, k))
    lib().orc_sptrsv(L.n_rows, _p(rp), _p(ci), _p(v), k, _p(B), _p(X))
    return X


def spmv_adj(A, X, G):
    """(GX, GV): GX = A^T G, GV[e] = sum_r G[i,r] X[col_e,r]."""
    rp, ci, v = _csr(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    k = G.shape[1] if G.ndim == 2 else 1
    GX = np.empty((A.n_cols, k))
    GV = np.empty(v.size)
    lib().orc_spmv_adj(A.n_rows, A.n_cols, _p(rp), _p(ci), _p(v), k, _p(X), _p(G), _p(GX), _p(GV))
    return GX, GV


def sptrsv_adj(L, X, G):
    """(GB, GV): L^T GB = G, GV[e] = -sum_r GB[i,r] X[col_e,r] (diagonal included)."""
    rp, ci, v = _csr(L)
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    k = G.shape[1] if G.ndim == 2 else 1
    GB = np.empty((L.n_rows, k))
    GV = np.empty(v.size)
    work = np.empty(L.n_rows * k)
    lib().orc_sptrsv_adj(L.n_rows, _p(rp), _p(ci), _p(v), k, _p(X), _p(G), _p(GB), _p(GV),
                         _p(work))
    return GB, GV


def levels(L):
    rp = np.ascontiguousarray(L.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(L.col_idx, dtype=np.int32)
    lev = np.zeros(max(L.n_rows, 1), dtype=np.int64)
    n = lib().orc_levels(L.n_rows, _p(rp), _p(ci), _p(lev))
    return lev[:L.n_rows], int(n)


def validate(kind, A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    return int(lib().orc_validate(kind, A.n_rows, A.n_cols, _p(rp), _p(ci)))


def transpose(A):
    """(AT, perm) with AT in CSR by a stable counting sort on column, perm[eT] = e."""
    from types import SimpleNamespace
    rp, ci, v = _csr(A)
    rpT = np.empty(A.n_cols + 1, dtype=np.int32)
    ciT = np.empty(ci.size, dtype=np.int32)
    vT = np.empty(ci.size)
    perm = np.empty(ci.size, dtype=np.int64)
    lib().orc_transpose(A.n_rows, A.n_cols, _p(rp), _p(ci), _p(v), _p(rpT), _p(ciT), _p(vT),
                        _p(perm))
    AT = SimpleNamespace(n_rows=A.n_cols, n_cols=A.n_rows, row_ptr=rpT, col_idx=ciT, values=vT)
    return AT, perm


def inspect(kind, A, t=64, sample=1, only_blas=False):
    """Canonical plan tables of Algorithm 1 for kind 0 (SpMV), 1 (lower solve, diagonal last)
    or 2 (transposed solve: upper, diagonal first, levels from the last row).  only_blas: the
    ablation's BLAS-only column-slice cover of every window."""
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    pp = lib().orc_inspect_ex(kind, A.n_rows, A.n_cols, _p(rp), _p(ci), t, sample, int(only_blas))
    try:
        p = pp.contents
        h = np.array(p.header[:], dtype=np.int64)
        npart, nreg, ncod, naux = (int(x) for x in h[5:9])

        def grab(ptr, n, dt):
            if n == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dt, copy=True)

        return {
            "header": h,
            "part_ptr": grab(p.part_ptr, npart + 1, np.int64),
            "part_rows": grab(p.part_rows, A.n_rows, np.int64),
            "regions": grab(p.regions, nreg * 8, np.int64).reshape(nreg, 8),
            "codelets": grab(p.codelets, ncod * 18, np.int64).reshape(ncod, 18),
            "aux": grab(p.aux, naux, np.int32),
        }
    finally:
        lib().orc_plan_free(pp)


def inspect_adjoint(kind, A, t=64, sample=1, only_blas=False):
    """Plan of the adjoint pass: for SpMV, A^T inspected as SpMV; for the lower solve,
    U = L^T (diagonal first) inspected as kind 2 on reverse levels.  Returns (plan, perm)."""
    AT, perm = transpose(A)
    return inspect(0 if kind == 0 else 2, AT, t, sample, only_blas), perm


def classify(kind, A, q):
    """(flags, nn) of candidate rows q (the explicit-FOPD classification)."""
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    q = np.ascontiguousarray(q, dtype=np.int64)
    nn = np.zeros(1, dtype=np.int64)
    f = lib().orc_classify(kind, _p(rp), _p(ci), _p(q), q.size, _p(nn))
    return int(f), int(nn[0])


_LIB_OMP = None


def lib_omp():
    """The many-core loops (ddf_oracle_omp.c)."""
    global _LIB_OMP
    if _LIB_OMP is None:
        path = os.path.join(_HERE, "liboracle_omp.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.omp_spmv.argtypes = [I32, P, P, P, I32, P, P]
        L.omp_spmv_adj.argtypes = [I32, I32, P, P, P, P, P, P, I32, P, P, P, P]
        L.omp_sptrsv.argtypes = [I32, P, P, P, I32, P, P, I64, P, P]
        L.omp_sptrsv_adj.argtypes = [I32, P, P, P, P, P, P, I32, P, P, I64, P, P, P, P]
        L.omp_threads.restype = I32
        _LIB_OMP = L
    return _LIB_OMP


def _reverse_cols(rpT, ciT, n):
    """Columns of the rows of a CSR pattern taken from the last row to the first, each column
    c renumbered n - 1 - c."""
    lens = np.diff(rpT)
    row_of = np.repeat(np.arange(n), lens)
    order = np.lexsort((np.arange(ciT.size), -row_of))
    return (n - 1 - ciT[order]).astype(np.int32)


def level_sets(lev, nlev):
    """(ptr[nlev + 1], rows) of the level sets, rows ascending within a level."""
    order = np.argsort(lev, kind="stable").astype(np.int64)
    ptr = np.zeros(nlev + 1, dtype=np.int64)
    np.cumsum(np.bincount(lev, minlength=nlev), out=ptr[1:])
    return ptr, order


def omp_threads():
    """Threads the many-core loops run on."""
    return int(lib_omp().omp_threads())


class ManyCore:
    """The serial oracle's value loops over host cores (OpenMP), for one matrix: the transposed
    pattern and the level sets are built once here (outside any timing)."""

    def __init__(self, A, triangular=False):
        self.A = A
        self.rp, self.ci, self.v = _csr(A)
        self.AT, perm = transpose(A)
        self.rpT = np.ascontiguousarray(self.AT.row_ptr, dtype=np.int32)
        self.ciT = np.ascontiguousarray(self.AT.col_idx, dtype=np.int32)
        self.perm = np.ascontiguousarray(perm, dtype=np.int64)
        if triangular:
            lev, nl = levels(A)
            self.lptr, self.lrows = level_sets(lev, nl)
            # reverse levels of U = L^T (0 for rows of U without off-diagonals, else one more
            # than the deepest of the later rows they read): the forward levels of U with its
            # rows and columns numbered from the end
            n = A.n_rows
            lens = np.diff(self.rpT)[::-1]
            rpR = np.zeros(n + 1, dtype=np.int32)
            np.cumsum(lens, out=rpR[1:])
            ciR = np.concatenate([n - 1 - self.ciT[self.rpT[i]:self.rpT[i + 1]] for i in range(n - 1, -1, -1)]) \
                if n < 4096 else _reverse_cols(self.rpT, self.ciT, n)
            from types import SimpleNamespace
            rl, nl = levels(SimpleNamespace(n_rows=n, row_ptr=rpR, col_idx=ciR.astype(np.int32), values=None))
            self.ulptr, self.ulrows = level_sets(rl[::-1].copy(), nl)

    def spmv(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        k = X.shape[1]
        Y = np.empty((self.A.n_rows, k))
        lib_omp().omp_spmv(self.A.n_rows, _p(self.rp), _p(self.ci), _p(self.v), k, _p(X), _p(Y))
        return Y

    def spmv_adj(self, X, G):
        X = np.ascontiguousarray(X, dtype=np.float64)
        G = np.ascontiguousarray(G, dtype=np.float64)
        k = G.shape[1]
        GX, GV = np.empty((self.A.n_cols, k)), np.empty(self.v.size)
        lib_omp().omp_spmv_adj(self.A.n_rows, self.A.n_cols, _p(self.rp), _p(self.ci), _p(self.v), _p(self.rpT),
                               _p(self.ciT), _p(self.perm), k, _p(X), _p(G), _p(GX), _p(GV))
        return GX, GV

    def sptrsv(self, B):
        B = np.ascontiguousarray(B, dtype=np.float64)
        k = B.shape[1]
        X = np.empty((self.A.n_rows, k))
        lib_omp().omp_sptrsv(self.A.n_rows, _p(self.rp), _p(self.ci), _p(self.v), k, _p(self.lptr),
                             _p(self.lrows), self.lptr.size - 1, _p(B), _p(X))
        return X

    def sptrsv_adj(self, X, G):
        X = np.ascontiguousarray(X, dtype=np.float64)
        G = np.ascontiguousarray(G, dtype=np.float64)
        k = G.shape[1]
        GB, GV = np.empty((self.A.n_rows, k)), np.empty(self.v.size)
        lib_omp().omp_sptrsv_adj(self.A.n_rows, _p(self.rp), _p(self.ci), _p(self.v), _p(self.rpT), _p(self.ciT),
                                 _p(self.perm), k, _p(self.ulptr), _p(self.ulrows), self.ulptr.size - 1, _p(X),
                                 _p(G), _p(GB), _p(GV))
        return GB, GV


def flags_count(flags):
    return ((flags & F_S0) != 0) + ((flags & F_S1) != 0) + ((flags & F_S2) != 0)
