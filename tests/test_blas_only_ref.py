"""The oracle's BLAS-only cover (the ablation of Sec. V-A and V-B: only BLAS codelets, as
column slices of rows, Sec. III-C) pinned to hand-derived covers and checked by brute force:
every codelet is BLAS on its explicit iteration space, the codelets cover every operation
exactly once, and the slices are the greedy cuts of each row."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from plan_decode import C, F_RECT, F_S0, F_S1, F_S2, F_SEP, decode_plan, expected_triples

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "psc_worked_example.json")
BLAS_FLAGS = F_S0 | F_S1 | F_S2 | F_SEP | F_RECT


def test_worked_example_blas_only():
    # Rows i = 0..2 hold columns {i, i+2, i+5}.  Each row cuts into {i, i+2} (stride 2) and
    # {i+5}; the three rows stack (row, value start and first column move by 1, 3, 1), so the
    # BLAS-only cover is a 3 x 2 codelet (sigma0 1, sigma1 2, cost 6 + 3) and a 3 x 1 codelet
    # at column 5 (cost 3 + 3): 15 in all, two codelets where the paper's example draws three
    # single-column ones (cost 18) - both are BLAS-only covers, the greedy cut is cheaper.
    g = json.load(open(GOLDEN))
    A = I.csr_from_pairs(g["n_rows"], g["n_cols"], np.array(g["rows"]), np.array(g["cols"]), np.arange(9.0))
    p = O.inspect(0, A, only_blas=True)
    assert p["regions"].tolist() == [[0, 0, 3, 0, 3, 15, 0, 0]]
    cod = p["codelets"]
    #                 type flags part reg u  m  nn P row0 rs op0 os col0 s0 s1 aux auxl cost
    assert cod.tolist() == [[0, BLAS_FLAGS, 0, 0, 0, 3, 2, 6, 0, 1, 0, 3, 0, 1, 2, 0, 0, 9],
                            [0, BLAS_FLAGS, 0, 0, 0, 3, 1, 3, 0, 1, 2, 3, 5, 1, 0, 0, 0, 6]]


def test_c1_interior_lines_blas_only():
    # 5-point Laplacian on 64 x 64, one window per grid line.  Inside an interior line
    # (j = 1..62) a row r holds {r-64, r-1, r, r+1, r+64}: cuts (0, w 2, stride 63),
    # (2, w 2, stride 1), (4, w 1); the first point {r-64, r, r+1, r+64}: (0, 2, 64),
    # (2, 2, 63); the last {r-64, r-1, r, r+64}: (0, 2, 63), (2, 2, 64).  Row by row:
    #   point 0: its two slices stack with nothing below (shapes differ): 2 + 3 and 2 + 3
    #   point 1: (0, 2, 63) stacks over points 1..63 (the last point has it too): 63*2 + 3
    #            (2, 2, 1) over points 1..62: 62*2 + 3;  (4, 1) over points 1..62: 62 + 3
    #   point 63: (2, 2, 64) alone: 2 + 3
    # -> costs [5, 5, 129, 127, 65, 5], 336 per interior line.
    p = O.inspect(0, I.c1_laplace2d().A, 64, only_blas=True)
    reg, cod = p["regions"], p["codelets"]
    assert np.all(reg[:, 4] == 3)
    for j in range(1, 63):
        mine = cod[cod[:, C["region"]] == j]
        assert mine[:, C["cost"]].tolist() == [5, 5, 129, 127, 65, 5], j
        assert mine[:, C["m"]].tolist() == [1, 1, 63, 62, 62, 1]
        assert reg[j, 5:8].tolist() == [336, 0, 0]


def test_bidiagonal_blas_only():
    # row 0 holds one op, row i >= 1 holds {i-1, i}: the first window is [m 1, m 63], every
    # other one a single 64-row codelet (the same cover as whole rows: every row is strided)
    n = 300
    rows = np.concatenate([np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(n - 1), np.arange(n)])
    A = I.csr_from_pairs(n, n, rows, cols, np.ones(rows.size))
    p = O.inspect(0, A, 64, only_blas=True)
    cod = p["codelets"]
    assert cod[cod[:, C["region"]] == 0][:, C["m"]].tolist() == [1, 63]
    for r in range(1, p["regions"].shape[0]):
        assert cod[cod[:, C["region"]] == r][:, C["m"]].tolist() == [p["regions"][r, 2]]


def greedy_cuts(cols):
    """(offset, width, stride) of a row's greedy strided cuts."""
    out, a, n = [], 0, cols.size
    while a < n:
        w, s = 1, 0
        if a + 1 < n:
            s = int(cols[a + 1] - cols[a])
            w = 2
            while a + w < n and cols[a + w] - cols[a + w - 1] == s:
                w += 1
        out.append((a, w, s if w >= 2 else 0))
        a += w
    return out


def check_blas_only(kind, A, p, t=64):
    cod = p["codelets"]
    assert np.array_equal(decode_plan(p), expected_triples(kind, A))
    assert np.all(cod[:, C["type"]] == 0) and np.all(cod[:, C["flags"]] == BLAS_FLAGS)
    assert np.all(cod[:, C["aux_len"]] == 0) and np.all(cod[:, C["cost"]] == cod[:, C["P"]] + 3)
    rp = A.row_ptr.astype(np.int64)
    off = 1 if kind == 2 else 0
    cut = 0 if kind == 0 else 1
    pp, pr, reg = p["part_ptr"], p["part_rows"], p["regions"]
    got_cuts = {}
    for rec in cod:
        r = reg[rec[C["region"]]]
        q = pr[pp[r[0]] + r[1] + rec[C["u"]]: pp[r[0]] + r[1] + rec[C["u"]] + rec[C["m"]]]
        m, w = int(rec[C["m"]]), int(rec[C["nn"]])
        a = int(rec[C["op0"]] - (rp[q[0]] + off))
        # brute force on the explicit iteration space: all three access functions strided
        f0 = np.repeat(q, w).reshape(m, w)
        f1 = (rp[q] + off + a)[:, None] + np.arange(w)[None, :]
        f2 = A.col_idx.astype(np.int64)[f1]

        def const(d):
            return d.size == 0 or bool(np.all(d == d.flat[0]))

        assert const(np.diff(f0[:, 0])) and const(np.diff(f1, axis=0)) and const(np.diff(f2, axis=0))
        assert const(np.diff(f2, axis=1))
        for row in q:
            got_cuts.setdefault(int(row), []).append((a, w, int(rec[C["sigma1"]])))
    for row in range(A.n_rows):
        b = rp[row] + off
        cols = A.col_idx[b:b + (rp[row + 1] - rp[row] - cut)].astype(np.int64)
        assert sorted(got_cuts.get(row, [])) == greedy_cuts(cols), row
    for ri, r in enumerate(reg):
        assert r[4] == 3 and r[5] == int(cod[cod[:, C["region"]] == ri][:, C["cost"]].sum())


@pytest.mark.parametrize("seed", range(8))
def test_random_blas_only(seed):
    rng = np.random.default_rng(40 + seed)
    A = I.random_csr(int(rng.integers(1, 200)), int(rng.integers(1, 200)), seed,
                     density=float(rng.uniform(0.01, 0.08)), runs=bool(seed % 2))
    check_blas_only(0, A, O.inspect(0, A, 16, only_blas=True), 16)
    L = I.random_lower(int(rng.integers(1, 200)), seed, density=0.04, runs=bool(seed % 2))
    check_blas_only(1, L, O.inspect(1, L, 64, only_blas=True))
    U, _ = O.transpose(L)
    check_blas_only(2, U, O.inspect(2, U, 64, only_blas=True))


def test_stencils_blas_only():
    w = I.c1_laplace2d()
    check_blas_only(0, w.A, O.inspect(0, w.A, only_blas=True))
    check_blas_only(1, w.L, O.inspect(1, w.L, only_blas=True))
    w = I.c5_laplace27(nx=8, k=1)
    check_blas_only(0, w.A, O.inspect(0, w.A, only_blas=True))


# ---- the library's column-slice schedule, replayed on the CPU ----
# Device record fields (16 int32) and the slice executor's rules: a task is rows [i0b, i0e) of
# one codelet; every (row, op) is added exactly once; in the solve a row is complete when all
# of its slices are in, and a slice may only read rows completed in earlier levels (tasks come
# in level order; a row with no ops is solved before the first level).
DF = {n: i for i, n in enumerate(["flags", "m", "nn", "row0", "row_step", "op0", "op_step", "col0", "sigma0",
                                  "sigma1", "rows_off", "ops_off", "cnt_off", "xt_off", "xp_off", "mat"])}


def replay_slices(kind, A, t):
    from paper_2111_12243_amd import ddf
    p = ddf.ddf_inspect(kind, A, ddf.ddf_opts_default(host_only=1, only_blas=1, window=t, build_adjoint=0))
    tabs = ddf.ddf_plan_device_tables(p, 0)
    canon = ddf.ddf_plan_export(p, 0)
    cods, tasks = tabs["cods"], tabs["tasks"]
    assert tabs["aux"].size == 0
    rp, ci = A.row_ptr.astype(np.int64), A.col_idx.astype(np.int64)
    x = np.random.default_rng(t).uniform(-1, 1, A.n_cols)
    y = np.zeros(A.n_rows)
    seen = np.zeros(A.nnz, np.int64)
    level = canon["codelets"][:, C["part"]]
    done_level = np.full(A.n_rows, -1)  # solve: level in which a row completed
    for tk in tasks:
        c = cods[tk[0]]
        assert c[DF["flags"]] & BLAS_FLAGS == BLAS_FLAGS and c[DF["rows_off"]] == -1
        assert 0 <= tk[1] < tk[2] <= c[DF["m"]]
        for i0 in range(tk[1], tk[2]):
            row = c[DF["row0"]] + i0 * c[DF["row_step"]]
            op = c[DF["op0"]] + i0 * c[DF["op_step"]]
            assert 0 <= row < A.n_rows
            for i1 in range(c[DF["nn"]]):
                e, col = op + i1, c[DF["col0"]] + i0 * c[DF["sigma0"]] + i1 * c[DF["sigma1"]]
                assert rp[row] <= e < rp[row + 1] and ci[e] == col
                if kind == 1:
                    assert e != rp[row + 1] - 1  # the diagonal is not an op
                    assert 0 <= done_level[col] < level[tk[0]] or rp[col + 1] - rp[col] == 1
                seen[e] += 1
                y[row] += A.values[e] * x[col]
        if kind == 1:
            # rows whose slices are all in by the end of this task's level
            for i0 in range(tk[1], tk[2]):
                row = c[DF["row0"]] + i0 * c[DF["row_step"]]
                diag = rp[row + 1] - 1
                if seen[rp[row]:diag].all():
                    done_level[row] = level[tk[0]]
    keep = np.ones(A.nnz, bool)
    if kind == 1:
        keep[rp[1:] - 1] = False
    assert (seen[keep] == 1).all() and (seen[~keep] == 0).all()
    if kind == 0:
        assert np.allclose(y, O.spmv(A, x[:, None])[:, 0], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_library_slice_schedule(seed):
    rng = np.random.default_rng(700 + seed)
    A = I.random_csr(int(rng.integers(1, 150)), int(rng.integers(1, 150)), seed, density=0.06, runs=bool(seed % 2))
    replay_slices(0, A, int(rng.choice([1, 8, 64])))
    L = I.random_lower(int(rng.integers(1, 150)), seed, density=0.05, runs=bool(seed % 2))
    replay_slices(1, L, int(rng.choice([1, 8, 64])))


def test_library_slice_schedule_workload():
    w = I.c5_laplace27(nx=8, k=1)
    replay_slices(0, w.A, 64)
    replay_slices(1, w.L, 64)
