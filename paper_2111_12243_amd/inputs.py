"""Seeded synthetic workloads: CSR matrices (int32 indices, FP64 values) and dense vectors.

This module only draws inputs.  It holds none of the arithmetic of the method (no products,
no solves, no inspection), so both the library path and the CPU oracle may take their inputs
from here.  Every workload is a pure function of its seed; draws happen in the order written
in each builder's docstring, with ``numpy.random.Generator(PCG64(seed))``.

The paper measures on SuiteSparse SPD matrices, which are not available here.  The stencil
workloads stand in for its FEM-like SPD matrices, the Chung-Lu power-law workload for its
irregular graph-like patterns, and the batch for a mix of both.

Grid rows are numbered ``r = i + nx*j + nx*ny*k`` (x fastest).
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 12243


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass
class CSR:
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int32 [n_rows+1]
    col_idx: np.ndarray  # int32 [nnz]
    values: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.n_rows >= 0 and self.row_ptr.size else 0

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.row_ptr, self.col_idx, self.values):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n_rows, self.n_cols))
        rows = np.repeat(np.arange(self.n_rows), np.diff(self.row_ptr))
        d[rows, self.col_idx] = self.values
        return d


def csr_from_pairs(n_rows: int, n_cols: int, rows: np.ndarray, cols: np.ndarray,
                   vals: np.ndarray | None = None) -> CSR:
    """Assemble a CSR from (row, col) pairs; pairs must be unique."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    counts = np.bincount(rows, minlength=n_rows)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    v = np.zeros(cols.size) if vals is None else np.asarray(vals, dtype=np.float64)[order]
    return CSR(n_rows, n_cols, rp.astype(np.int32), cols.astype(np.int32), v)


def dense_to_csr(d: np.ndarray) -> CSR:
    r, c = np.nonzero(d)
    return csr_from_pairs(d.shape[0], d.shape[1], r, c, d[r, c])


def tril(a: CSR) -> CSR:
    """Entries with col <= row, diagonal included (pattern and values copied)."""
    rows = np.repeat(np.arange(a.n_rows, dtype=np.int64), np.diff(a.row_ptr))
    keep = a.col_idx.astype(np.int64) <= rows
    counts = np.bincount(rows[keep], minlength=a.n_rows)
    rp = np.zeros(a.n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return CSR(a.n_rows, a.n_rows, rp.astype(np.int32), a.col_idx[keep].copy(), a.values[keep].copy())


# ----------------------------------------------------------------------------------------
# stencils
# ----------------------------------------------------------------------------------------

OFFS_5PT = [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)]
OFFS_27PT = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def stencil_pattern(nx: int, ny: int, nz: int, offs, n: int | None = None):
    """CSR pattern of a stencil on an nx*ny*nz grid, restricted to its first n rows/cols.

    ``offs`` are (dx, dy, dz) sorted by (dz, dy, dx), which is increasing column order.
    Returns (row_ptr int64, col_idx int32, offset_id int8).
    """
    N = nx * ny * nz
    n = N if n is None else int(n)
    r = np.arange(n, dtype=np.int64)
    i = r % nx
    j = (r // nx) % ny
    k = r // (nx * ny)
    masks = []
    for dx, dy, dz in offs:
        ok = ((i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny)
              & (k + dz >= 0) & (k + dz < nz))
        ok &= (r + dx + nx * dy + nx * ny * dz) < n
        masks.append(ok)
    counts = np.zeros(n, dtype=np.int64)
    for ok in masks:
        counts += ok
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    nnz = int(rp[-1])
    col = np.empty(nnz, dtype=np.int32)
    oid = np.empty(nnz, dtype=np.int8)
    cur = rp[:-1].copy()
    for o, ((dx, dy, dz), ok) in enumerate(zip(offs, masks)):
        pos = cur[ok]
        col[pos] = (r[ok] + dx + nx * dy + nx * ny * dz).astype(np.int32)
        oid[pos] = o
        cur[ok] += 1
    return rp, col, oid


def laplacian(nx: int, ny: int, nz: int, offs, diag: float, off: float = -1.0) -> CSR:
    rp, col, oid = stencil_pattern(nx, ny, nz, offs)
    n = nx * ny * nz
    center = offs.index((0, 0, 0))
    vals = np.full(col.size, off, dtype=np.float64)
    vals[oid == center] = diag
    return CSR(n, n, rp.astype(np.int32), col, vals)


def lower_offsets(offs):
    return [o for o in offs if (o[2], o[1], o[0]) <= (0, 0, 0)]


# ----------------------------------------------------------------------------------------
# Chung-Lu power-law rows built from runs of consecutive columns
# ----------------------------------------------------------------------------------------

def chung_lu_expected(n: int, gamma: float, mean_deg: float, rng: np.random.Generator):
    """Expected degrees e_i = min(c*w_i, cap), w = (rank+1)^(-1/(gamma-1)) through a seeded
    permutation, cap = sqrt(mean_deg*n), c by bisection so that sum(e) = mean_deg*n.
    Draws: one permutation of n."""
    w_rank = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    perm = rng.permutation(n)
    w = np.empty(n)
    w[perm] = w_rank
    cap = math.sqrt(mean_deg * n)
    target = mean_deg * n
    lo, hi = 0.0, target / w.min()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = np.minimum(mid * w, cap).sum()
        if s < target:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * w, cap)


def run_rows(n_rows: int, deg: np.ndarray, start_cdf: np.ndarray, rng: np.random.Generator,
             limit: np.ndarray, lmin: int = 4, lmax: int = 32):
    """Rows made of runs of consecutive columns.

    For each row, run lengths L ~ U{lmin..lmax} are drawn until the drawn lengths reach the
    row's degree (the last one truncated to what remains).  Each run start is a node drawn
    with probability proportional to ``start_cdf`` (a cumulative weight table over
    [0, len(start_cdf))), scaled into [0, limit_i) and clipped to [0, limit_i - L].  Runs of a
    row are merged (set union), so overlapping runs give a row fewer than ``deg`` entries.
    Draws: run lengths (sum of ceil(deg/lmin)), then one uniform per kept run.
    Returns (rows int64, cols int64) of unique pairs."""
    deg = np.minimum(deg.astype(np.int64), limit.astype(np.int64))
    maxruns = (deg + lmin - 1) // lmin
    tot = int(maxruns.sum())
    lens = rng.integers(lmin, lmax + 1, size=tot).astype(np.int64)
    row_of = np.repeat(np.arange(n_rows, dtype=np.int64), maxruns)
    seg0 = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(maxruns, out=seg0[1:])
    cs = np.cumsum(lens)
    before = cs - lens - np.repeat(np.concatenate(([0], cs))[seg0[:-1]], maxruns)
    keep = before < deg[row_of]
    row_of = row_of[keep]
    leff = np.minimum(lens[keep], deg[row_of] - before[keep])
    u = rng.random(row_of.size)
    node = np.searchsorted(start_cdf, u * start_cdf[-1], side="right")
    node = np.minimum(node, start_cdf.size - 1)
    lim = limit[row_of].astype(np.int64)
    start = (node.astype(np.float64) * lim / start_cdf.size).astype(np.int64)
    start = np.clip(start, 0, np.maximum(lim - leff, 0))
    r = np.repeat(row_of, leff)
    within = np.arange(r.size, dtype=np.int64) - np.repeat(np.cumsum(leff) - leff, leff)
    c = np.repeat(start, leff) + within
    key = np.unique(r * int(limit.max() + 1) + c)
    return key // int(limit.max() + 1), key % int(limit.max() + 1)


# ----------------------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    A: CSR | None = None  # SpMV matrix
    L: CSR | None = None  # lower-triangular matrix (diagonal last in each row)
    k: int = 1
    X: np.ndarray | None = None  # SpMV input (n_cols, k)
    Gy: np.ndarray | None = None  # SpMV upstream gradient (n_rows, k)
    B: np.ndarray | None = None  # SpTRSV right-hand side (n, k)
    Gx: np.ndarray | None = None  # SpTRSV upstream gradient (n, k)
    batch: list = field(default_factory=list)  # batch workloads: list of dicts {L, k, B, G}
    meta: dict = field(default_factory=dict)


def _u(rng, shape):
    return rng.uniform(-1.0, 1.0, size=shape)


def c1_laplace2d(nx: int = 64) -> Workload:
    """5-point Laplacian on nx*nx (diag 4, neighbours -1); L = tril(A); k = 1.
    Draws (seed 12244): X (n,1), Gy (n,1), B (n,1), Gx (n,1), all U[-1,1]."""
    rng = generator(SEED_BASE + 1)
    A = laplacian(nx, nx, 1, OFFS_5PT, 4.0)
    n = A.n_rows
    w = Workload("c1_laplace2d_64x64", A=A, L=tril(A), k=1)
    w.X, w.Gy, w.B, w.Gx = _u(rng, (n, 1)), _u(rng, (n, 1)), _u(rng, (n, 1)), _u(rng, (n, 1))
    return w


def c2_stencil27_offband(nx: int = 100, n_rand: int = 4) -> Workload:
    """27-point stencil on nx^3, off-diagonals U[-1,1], plus n_rand columns per row drawn
    uniformly without replacement from {c : |c - r| > nx*nx + nx + 1} (outside the stencil
    band).  Diagonal = 1 + sum over the full row of |A_rc|.  L = tril(A).  k = 1.
    Draws (seed 12245): random columns (n, n_rand) with re-draws of rows holding a repeat,
    off-diagonal values U[-1,1] over all nnz in CSR order, then X, Gy, B, Gx (n,1)."""
    rng = generator(SEED_BASE + 2)
    n = nx * nx * nx
    band = nx * nx + nx + 1
    rp, col, oid = stencil_pattern(nx, nx, nx, OFFS_27PT)
    r = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, r - band)
    hi = np.minimum(n - 1, r + band)
    width = hi - lo + 1
    count = n - width
    draws = rng.integers(0, count[:, None], size=(n, n_rand))
    while True:
        s = np.sort(draws, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            break
        draws[bad] = rng.integers(0, count[bad, None], size=(bad.size, n_rand))
    rc = np.where(draws < lo[:, None], draws, draws + width[:, None])
    srow = np.repeat(r, np.diff(rp))
    rows = np.concatenate([srow, np.repeat(r, n_rand)])
    cols = np.concatenate([col.astype(np.int64), rc.ravel()])
    A = csr_from_pairs(n, n, rows, cols)
    A.values = _u(rng, A.nnz)
    arow = np.repeat(r, np.diff(A.row_ptr.astype(np.int64)))
    isdiag = A.col_idx.astype(np.int64) == arow
    off = np.where(isdiag, 0.0, np.abs(A.values))
    rowsum = np.bincount(arow, weights=off, minlength=n)
    A.values[isdiag] = 1.0 + rowsum
    w = Workload(f"c2_stencil27_{nx}^3_offband{n_rand}", A=A, L=tril(A), k=1)
    w.X, w.Gy, w.B, w.Gx = _u(rng, (n, 1)), _u(rng, (n, 1)), _u(rng, (n, 1)), _u(rng, (n, 1))
    return w


def c3_chung_lu(n: int = 4_000_000, mean_deg: float = 16.0, gamma: float = 2.1) -> Workload:
    """Chung-Lu power-law rows (gamma 2.1, mean degree 16, cap sqrt(16 n)), each row made of
    runs of consecutive columns of length U{4..32} whose starts are drawn proportionally to
    the capped weights.  d_i = max(1, floor(e_i + U[0,1))).  Values N(0,1).  SpMV only.
    Draws (seed 12246): weight permutation, n uniforms for d, run lengths, run starts,
    values N(0,1) over nnz, then X, Gy (n,1) U[-1,1]."""
    rng = generator(SEED_BASE + 3)
    e = chung_lu_expected(n, gamma, mean_deg, rng)
    d = np.maximum(1, np.floor(e + rng.random(n))).astype(np.int64)
    cdf = np.cumsum(e)
    rows, cols = run_rows(n, d, cdf, rng, np.full(n, n, dtype=np.int64))
    A = csr_from_pairs(n, n, rows, cols)
    A.values = rng.standard_normal(A.nnz)
    w = Workload(f"c3_chung_lu_n{n}", A=A, k=1)
    w.X, w.Gy = _u(rng, (n, 1)), _u(rng, (n, 1))
    w.meta["max_row"] = int(np.diff(A.row_ptr).max())
    return w


def _lower_from_pattern(rp, col, rng) -> CSR:
    """Off-diagonal values U[-1,1]; diagonal = 1 + row abs-sum.  Pattern must hold the
    diagonal as the last entry of every row."""
    n = rp.size - 1
    vals = _u(rng, col.size)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    isdiag = col.astype(np.int64) == rows
    rowsum = np.bincount(rows, weights=np.where(isdiag, 0.0, np.abs(vals)), minlength=n)
    vals[isdiag] = 1.0 + rowsum
    return CSR(n, n, rp.astype(np.int32), col.astype(np.int32), vals)


def batch_matrix(b: int, n_lo: float = 1e3, n_hi: float = 2e5, kmax: int = 32) -> dict:
    """Matrix b of the batch (seed 12247*1000 + b).
    Draws: n_b = round(exp(U[ln n_lo, ln n_hi])), k_b ~ U{1..kmax}, then the pattern's own
    draws (kind 2 only), off-diagonal values U[-1,1], then B, G (n_b, k_b) U[-1,1].
    Kind b mod 3: 0 = 2D 5-point lower on a ceil(sqrt n)-wide grid; 1 = 3D 27-point lower on
    ceil(cbrt n)^2 planes; 2 = power-law lower rows (Chung-Lu, mean 8 off-diagonals, runs
    of consecutive columns below the diagonal)."""
    rng = generator((SEED_BASE + 4) * 1000 + b)
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    k = int(rng.integers(1, kmax + 1))
    kind = b % 3
    if kind == 0:
        wdt = int(math.ceil(math.sqrt(n)))
        rp, col, _ = stencil_pattern(wdt, (n + wdt - 1) // wdt, 1, lower_offsets(OFFS_5PT), n)
    elif kind == 1:
        wdt = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
        rp, col, _ = stencil_pattern(wdt, wdt, (n + wdt * wdt - 1) // (wdt * wdt),
                                     lower_offsets(OFFS_27PT), n)
    else:
        e = chung_lu_expected(n, 2.1, 8.0, rng)
        d = np.floor(e + rng.random(n)).astype(np.int64)
        limit = np.arange(n, dtype=np.int64)  # columns < i
        rows, cols = run_rows(n, d, np.cumsum(e), rng, np.maximum(limit, 1))
        keep = cols < rows
        rows, cols = rows[keep], cols[keep]
        rows = np.concatenate([rows, np.arange(n, dtype=np.int64)])
        cols = np.concatenate([cols, np.arange(n, dtype=np.int64)])
        t = csr_from_pairs(n, n, rows, cols)
        rp, col = t.row_ptr.astype(np.int64), t.col_idx
    L = _lower_from_pattern(rp, col, rng)
    return {"L": L, "k": k, "kind": kind, "B": _u(rng, (n, k)), "G": _u(rng, (n, k))}


def c4_batch(nmat: int = 256, **kw) -> Workload:
    w = Workload(f"c4_batch{nmat}")
    w.batch = [batch_matrix(b, **kw) for b in range(nmat)]
    return w


def c5_laplace27(nx: int = 170, k: int = 8) -> Workload:
    """27-point Laplacian on nx^3 (off-diagonals -1, diagonal 26); L = tril(A); k RHS.
    Draws (seed 12248): X, Gy, B, Gx (n,k) U[-1,1]."""
    rng = generator(SEED_BASE + 5)
    A = laplacian(nx, nx, nx, OFFS_27PT, 26.0)
    n = A.n_rows
    w = Workload(f"c5_laplace27_{nx}^3_k{k}", A=A, L=tril(A), k=k)
    w.X, w.Gy, w.B, w.Gx = _u(rng, (n, k)), _u(rng, (n, k)), _u(rng, (n, k)), _u(rng, (n, k))
    return w


WORKLOADS = {"c1": c1_laplace2d, "c2": c2_stencil27_offband, "c3": c3_chung_lu,
             "c4": c4_batch, "c5": c5_laplace27}


def workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)


# ----------------------------------------------------------------------------------------
# small random patterns for tests
# ----------------------------------------------------------------------------------------

def random_csr(n_rows: int, n_cols: int, seed: int, density: float = 0.1,
               empty_frac: float = 0.1, runs: bool = False) -> CSR:
    """Random pattern with some empty rows; with runs=True rows are built from short runs."""
    rng = generator(seed)
    rows, cols = [], []
    for i in range(n_rows):
        if rng.random() < empty_frac or n_cols == 0:
            continue
        if runs:
            c = set()
            for _ in range(int(rng.integers(1, 4))):
                s = int(rng.integers(0, n_cols))
                c.update(range(s, min(n_cols, s + int(rng.integers(1, 9)))))
            c = np.array(sorted(c), dtype=np.int64)
        else:
            c = np.nonzero(rng.random(n_cols) < density)[0]
        rows.append(np.full(c.size, i))
        cols.append(c)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    a = csr_from_pairs(n_rows, n_cols, rows, cols)
    a.values = rng.uniform(-1, 1, a.nnz)
    return a


def long_rows_lower(n: int = 600, seed: int = 5) -> CSR:
    """Sparse random lower-triangular matrix plus a few rows of hundreds of entries: a full
    prefix (one run), a strided row, two scattered rows, and a dense first column (a long row
    of the transpose).  Off-diagonals U[-0.01, 0.01], diagonal 1 + U[0, 1]."""
    rng = generator(seed)
    base = random_lower(n, seed, density=0.004)
    r, c = [], []
    for i in range(n):
        cols = base.col_idx[base.row_ptr[i]:base.row_ptr[i + 1]]
        r.append(np.full(cols.size, i))
        c.append(cols)
    h, s = n // 2, (5 * n) // 6
    extra = {h: np.arange(h), h + 1: rng.choice(h + 1, (5 * n) // 12, replace=False), s: np.arange(0, s, 3),
             n - 1: rng.choice(n - 1, (2 * n) // 3, replace=False)}
    for i, cols in extra.items():
        r.append(np.full(cols.size, i))
        c.append(cols)
    r.append(np.arange(1, n))
    c.append(np.zeros(n - 1, np.int64))
    rows, cols = np.concatenate(r), np.concatenate(c)
    pairs = np.unique(np.stack([rows, cols], 1), axis=0)
    rows, cols = pairs[:, 0], pairs[:, 1]
    off = cols < rows
    vals = rng.uniform(-1, 1, rows.size) * 0.01
    vals[~off] = 1.0 + rng.uniform(0, 1, (~off).sum())
    return csr_from_pairs(n, n, rows, cols, vals)


def random_lower(n: int, seed: int, density: float = 0.2, runs: bool = False) -> CSR:
    """Random lower-triangular matrix, diagonal = 1 + row abs-sum (last in each row)."""
    rng = generator(seed)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for i in range(1, n):
        if runs:
            c = set()
            for _ in range(int(rng.integers(0, 3))):
                s = int(rng.integers(0, i))
                c.update(range(s, min(i, s + int(rng.integers(1, 6)))))
            c = np.array(sorted(c), dtype=np.int64)
        else:
            c = np.nonzero(rng.random(i) < density)[0]
        rows.append(np.full(c.size, i))
        cols.append(c)
    t = csr_from_pairs(n, n, np.concatenate(rows), np.concatenate(cols))
    return _lower_from_pattern(t.row_ptr.astype(np.int64), t.col_idx, rng)


def mixed_lower(n: int, seed: int, long_every: int = 150, long_ops: int = 8, short_max: int = 3) -> CSR:
    """Lower-triangular matrix of short rows (0..short_max random earlier columns) with every
    long_every-th row holding long_ops; diagonal = 1 + row abs-sum (last in each row)."""
    rng = generator(seed)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for i in range(1, n):
        k = min(i, long_ops if i % long_every == 0 else int(rng.integers(0, short_max + 1)))
        c = np.sort(rng.choice(i, size=k, replace=False)) if k else np.zeros(0, np.int64)
        rows.append(np.full(c.size, i))
        cols.append(c)
    t = csr_from_pairs(n, n, np.concatenate(rows), np.concatenate(cols))
    return _lower_from_pattern(t.row_ptr.astype(np.int64), t.col_idx, rng)


def hub_lower(n: int, seed: int, hub_every: int = 97, hub_ops: int = 30, near: int = 50, far: int = 300) -> CSR:
    """Lower-triangular chain (row i reads row i-1, plus up to two random columns among the
    `near` rows before it) with every hub_every-th row also reading hub_ops random columns at
    least `far` rows back; diagonal = 1 + row abs-sum (last in each row)."""
    rng = generator(seed)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for i in range(1, n):
        c = {i - 1}
        lo = max(0, i - near)
        for _ in range(int(rng.integers(0, 3))):
            if i - 1 > lo:
                c.add(int(rng.integers(lo, i - 1)))
        if i % hub_every == 0 and i > far + hub_ops:
            c.update(int(x) for x in rng.choice(i - far, size=hub_ops, replace=False))
        c = np.array(sorted(c), dtype=np.int64)
        rows.append(np.full(c.size, i))
        cols.append(c)
    t = csr_from_pairs(n, n, np.concatenate(rows), np.concatenate(cols))
    return _lower_from_pattern(t.row_ptr.astype(np.int64), t.col_idx, rng)


def cached(name: str, builder, *args, **kw):
    """Build a workload once per process (and optionally on disk when DDF_INPUT_CACHE is set)."""
    key = (name, args, tuple(sorted(kw.items())))
    if key in _MEMO:
        return _MEMO[key]
    w = builder(*args, **kw)
    _MEMO[key] = w
    return w


_MEMO: dict = {}
