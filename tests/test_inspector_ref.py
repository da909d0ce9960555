"""The oracle inspector (Algorithm 1 with the FOPD classification and Eq. (1)) pinned to the
paper's worked example, hand-derived plans, definition-level brute force and invariants."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from plan_decode import (C, F_RECT, F_RUNS, F_S0, F_S1, F_S2, F_SEP, codelet_rows, decode_plan,
                         expected_triples)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "psc_worked_example.json")


def worked_example():
    g = json.load(open(GOLDEN))
    vals = np.arange(float(len(g["cols"])))
    return I.csr_from_pairs(g["n_rows"], g["n_cols"], np.array(g["rows"]), np.array(g["cols"]), vals)


def test_paper_worked_example():
    e = json.load(open(GOLDEN))["expect"]
    p = O.inspect(0, worked_example())
    assert p["codelets"].shape == (1, 18)
    c = dict(zip(O.COD_FIELDS, p["codelets"][0]))
    assert c["type"] == e["type"]  # PSC I: f0 and f1 strided, h (x) not
    assert c["flags"] == F_S0 | F_S1 | F_SEP | F_RECT
    assert c["op_step"] == e["op_step"]  # FOPD_i0 of g = 3, FOPD_i1 = 1
    assert c["sigma0"] == e["sigma0"]
    assert list(p["aux"]) == e["offsets"]  # the shared offset table s
    # h needs |s| + 1 = 4 loads; Eq. (1): 9 ops + 3 functions + 3 table entries
    assert c["cost"] == e["cost"]
    # a 3-BLAS cover would cost 3 * (3 + 3) = 18 > 15, and needs 9 loads (3 per codelet)
    assert p["regions"][0, 5:].tolist() == e["region_costs"]


def test_worked_example_fopd():
    A = worked_example()
    # Delta_{i1} h(1,1) = h(1,2) - h(1,1) = 6 - 3 = 3: h is not strided
    assert A.col_idx[5] - A.col_idx[4] == 3
    fl, nn = O.classify(0, A, np.arange(3))
    assert nn == 3 and fl & F_S0 and fl & F_S1 and not fl & F_S2


def test_identity_plan():
    n, t = 200, 64
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.ones(n))
    p = O.inspect(0, eye, t)
    cod = p["codelets"]
    assert cod.shape[0] == (n + t - 1) // t
    assert np.all(cod[:, C["type"]] == 0)
    assert cod[:, C["m"]].tolist() == [64, 64, 64, 8]
    assert p["aux"].size == 0


def bidiag(n):
    rows = np.concatenate([np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(n - 1), np.arange(n)])
    return I.csr_from_pairs(n, n, rows, cols, np.ones(rows.size))


def test_bidiagonal_spmv_plan():
    n, t = 300, 64
    p = O.inspect(0, bidiag(n), t)
    reg, cod = p["regions"], p["codelets"]
    assert np.all(cod[:, C["type"]] == 0)
    first = cod[cod[:, C["region"]] == 0]
    assert first[:, C["m"]].tolist() == [1, t - 1]
    for r in range(1, reg.shape[0]):
        rc = cod[cod[:, C["region"]] == r]
        assert rc.shape[0] == 1 and rc[0, C["m"]] == reg[r, 2]


def test_bidiagonal_sptrsv_plan():
    n = 50
    p = O.inspect(1, bidiag(n))
    assert p["header"][5] == n
    cod = p["codelets"]
    assert cod.shape[0] == n and np.all(cod[:, C["type"]] == 0) and np.all(cod[:, C["m"]] == 1)


def test_c1_spmv_plan():
    p = O.inspect(0, I.c1_laplace2d().A, 64)
    cod = p["codelets"]
    assert cod.shape[0] == 192 and np.all(cod[:, C["type"]] == 1)
    costs = cod[:, C["cost"]].reshape(64, 3)
    assert costs[0].tolist() == [9, 255, 9] and costs[-1].tolist() == [9, 255, 9]
    assert np.all(costs[1:-1] == [11, 318, 11])
    assert int(cod[:, C["cost"]].sum()) == 21626


def test_c1_sptrsv_plan():
    p = O.inspect(1, I.c1_laplace2d().L, 64)
    cod = p["codelets"]
    assert p["header"][5] == 127
    assert cod.shape[0] == 251 and np.all(cod[:, C["type"]] == 0)
    assert int(cod[:, C["P"]].sum()) == 8064
    assert int(cod[:, C["cost"]].sum()) == 8817


def test_c1_spmv_region_costs():
    # Each window is one grid line of 64 points (Eq. 1, c = |p| + 3 + |s0| + |s1| + |s2|).
    # BLAS_first = PSCI_first: no single row is BLAS (its columns are not one stride), so both
    # take the longest PSC I runs: the edge point, the 62 interior points, the other edge point.
    #   boundary line j = 0 or 63: rows of 3, 4 x 62, 3 entries -> (3+3+3) + (248+3+4) + (3+3+3)
    #     = 273; the shared pattern {0, 1, 2, 65} of the middle codelet has 2 runs, and 2*2 = 4
    #     ties its 4 plain offsets, so it stays PLAIN (ties go to the plain table)
    #   interior line: rows of 4, 5 x 62, 4 -> (4+3+4) + (310+3+5) + (4+3+4) = 340
    # PSCII_first takes the whole ragged line as one PSC II codelet (only the rows are strided):
    # |p| + 3 + 64 op starts + |p| plain columns (runs would cost 2 * 3 per row, more than |p|):
    #   boundary: 254 + 3 + 64 + 254 = 575;  interior: 318 + 3 + 64 + 318 = 703
    p = O.inspect(0, I.c1_laplace2d().A, 64)
    reg = p["regions"]
    assert reg.shape[0] == 64
    for j in range(64):
        want = [273, 273, 575] if j in (0, 63) else [340, 340, 703]
        assert reg[j, 5:8].tolist() == want, j
        assert reg[j, 4] == 0  # the tie goes to BLAS_first
    assert not np.any(p["codelets"][:, C["flags"]] & F_RUNS)


def _rows_csr(cols_per_row, n_cols):
    rows = np.concatenate([np.full(len(c), i) for i, c in enumerate(cols_per_row)])
    cols = np.concatenate([np.asarray(c) for c in cols_per_row])
    return I.csr_from_pairs(len(cols_per_row), n_cols, rows, cols, np.ones(rows.size))


def test_runs_table_strictly_smaller():
    # Row q holds {q..q+3} and {q+10..q+13}: rectangular, rows and value offsets strided,
    # separable (sigma0 = 1), columns not strided -> one PSC I codelet over the 4 rows.  Its
    # shared pattern {0,1,2,3,10,11,12,13} has R = 2 runs: 2R = 4 < 8 plain offsets, so the
    # table is runs (0, 4), (10, 4) and the cost is 32 + 3 + 4 = 39 for every strategy.
    A = _rows_csr([np.r_[q:q + 4, q + 10:q + 14] for q in range(4)], 20)
    p = O.inspect(0, A, 64)
    assert p["codelets"].shape[0] == 1
    c = dict(zip(O.COD_FIELDS, p["codelets"][0]))
    assert c["flags"] == F_S0 | F_S1 | F_SEP | F_RECT | F_RUNS and c["type"] == 1
    assert c["sigma0"] == 1 and c["col0"] == 0
    assert p["aux"].tolist() == [0, 4, 10, 4]
    assert c["cost"] == 39 and p["regions"][0, 4:8].tolist() == [0, 39, 39, 39]


def test_runs_table_tie_stays_plain():
    # Row q holds {q, q+1, q+5, q+6}: the shared pattern {0, 1, 5, 6} has R = 2 runs, and
    # 2R = 4 equals its 4 plain offsets: the tie keeps the plain table.  Cost 16 + 3 + 4 = 23.
    A = _rows_csr([[q, q + 1, q + 5, q + 6] for q in range(4)], 12)
    p = O.inspect(0, A, 64)
    c = dict(zip(O.COD_FIELDS, p["codelets"][0]))
    assert c["flags"] == F_S0 | F_S1 | F_SEP | F_RECT
    assert p["aux"].tolist() == [0, 1, 5, 6] and c["cost"] == 23


def test_runs_full_table():
    # Two rows {0..3, 10..13} and {1..4, 15..18}: rectangular (8 each), not separable (the
    # column difference between the rows is 1 for the first run and 5 for the second).  PSC I
    # with a full column table: 16 plain columns against R = 4 runs -> 2R = 8 < 16, runs
    # (start, len) per row.  Cost 16 + 3 + 8 = 27; two single-row codelets would cost 2 * 15.
    A = _rows_csr([np.r_[0:4, 10:14], np.r_[1:5, 15:19]], 20)
    p = O.inspect(0, A, 64)
    assert p["codelets"].shape[0] == 1
    c = dict(zip(O.COD_FIELDS, p["codelets"][0]))
    assert c["flags"] == F_S0 | F_S1 | F_RECT | F_RUNS and c["type"] == 1
    assert p["aux"].tolist() == [0, 4, 10, 4, 1, 4, 15, 4] and c["cost"] == 27


def test_pscii_first_strictly_cheapest():
    # Rows of 5, 6, 5, 6 entries, each two runs: {q, q+1} and 3 or 4 columns from q+10.
    # A single row is PSC I (its columns have strides 1, 9, 1 ...) and any two neighbours are
    # ragged (only the rows stay strided), so BLAS_first and PSCI_first both cut one codelet
    # per row, each with a shared pattern of R = 2 runs (2R = 4 < 5 or 6 offsets):
    #   (5+3+4) + (6+3+4) + (5+3+4) + (6+3+4) = 50.
    # PSCII_first keeps the 4 rows together (rows strided): |p| = 22, + 3, + 4 op starts, and
    # full runs, 2 per row: 2 * 8 = 16 < 22 plain columns -> 22 + 3 + 4 + 16 = 45 (row counts
    # are loop bounds, not costed).  PSCII_first is strictly cheapest and is chosen.
    rows = [np.r_[q:q + 2, q + 10:q + 13 + (q % 2)] for q in range(4)]
    A = _rows_csr(rows, 20)
    p = O.inspect(0, A, 64)
    reg = p["regions"][0]
    assert reg[4:8].tolist() == [2, 50, 50, 45]
    assert p["codelets"].shape[0] == 1
    c = dict(zip(O.COD_FIELDS, p["codelets"][0]))
    assert c["type"] == 2 and c["flags"] == F_S0 | F_RUNS and c["nn"] == -1 and c["cost"] == 45
    # OPSTART, COUNTS, then the runs of each row (start, len)
    assert p["aux"].tolist() == [0, 5, 11, 16, 5, 6, 5, 6,
                                 0, 2, 10, 3, 1, 2, 11, 4, 2, 2, 12, 3, 3, 2, 13, 4]


# ---------------------------------------------------------------- brute force + invariants

def brute_flags(kind, A, rows):
    """FOPD flags recomputed from the explicit iteration space with numpy."""
    rp = A.row_ptr.astype(np.int64)
    off = 1 if kind == 2 else 0
    ln = np.diff(rp)[rows] - (0 if kind == 0 else 1)
    rect = bool(np.all(ln == ln[0]))
    dq = np.diff(rows)
    s0 = dq.size <= 1 or bool(np.all(dq == dq[0]))
    if not rect:
        return (F_S0 if s0 else 0)
    nn = int(ln[0])
    I0 = np.repeat(np.arange(rows.size), nn).reshape(rows.size, nn)
    I1 = np.tile(np.arange(nn), rows.size).reshape(rows.size, nn)
    f1 = rp[rows][I0] + off + I1
    f2 = A.col_idx.astype(np.int64)[f1] if nn else f1

    def const(d):
        return d.size == 0 or bool(np.all(d == d.flat[0]))

    s1 = const(np.diff(f1, axis=0))
    sep = const(np.diff(f2, axis=0))
    s2 = sep and const(np.diff(f2, axis=1))
    return ((F_S0 if s0 else 0) | (F_S1 if s1 else 0) | (F_S2 if s2 else 0)
            | (F_SEP if sep else 0) | F_RECT)


def brute_runs(kind, A, q, fl):
    """The column table is stored as runs when 2 x (maximal runs of consecutive columns) is
    below its plain size: the shared pattern's nn offsets (SEP) or every column."""
    if fl & F_S2:
        return False
    rp = A.row_ptr.astype(np.int64)
    off = 1 if kind == 2 else 0
    cut = 0 if kind == 0 else 1

    def cols(r):
        b = rp[r] + off
        return A.col_idx[b:b + (rp[r + 1] - rp[r] - cut)].astype(np.int64)

    def runs(c):
        return 0 if c.size == 0 else 1 + int(np.count_nonzero(np.diff(c) != 1))

    if fl & F_SEP:
        c = cols(q[0])
        return 2 * runs(c) < c.size
    cs = [cols(r) for r in q]
    return 2 * sum(runs(c) for c in cs) < sum(c.size for c in cs)


def check_plan(kind, A, p, t=64):
    cod, reg = p["codelets"], p["regions"]
    # exact cover: decoding the plan reproduces the operations of the CSR
    got = decode_plan(p)
    exp = expected_triples(kind, A)
    assert np.array_equal(got, exp)
    rows = codelet_rows(p)
    assert np.array_equal(np.sort(rows), np.arange(A.n_rows))
    # codelets stay inside their region and partition; positions follow part_rows
    pp, pr = p["part_ptr"], p["part_rows"]
    for rec in cod:
        r = reg[rec[C["region"]]]
        assert rec[C["part"]] == r[0]
        u, m = rec[C["u"]], rec[C["m"]]
        assert 0 <= u and u + m <= r[2]
        q = pr[pp[r[0]] + r[1] + u: pp[r[0]] + r[1] + u + m]
        fl = brute_flags(kind, A, q)
        assert (rec[C["flags"]] & ~F_RUNS) == fl
        assert bool(rec[C["flags"]] & F_RUNS) == brute_runs(kind, A, q, fl)
        k = ((fl & F_S0) != 0) + ((fl & F_S1) != 0) + ((fl & F_S2) != 0)
        assert rec[C["type"]] == 3 - k
    # the chosen strategy is the cheapest, ties to the first; its codelets add up to it
    for ri, r in enumerate(reg):
        if r[4] < 0:
            continue
        costs = r[5:8]
        assert r[4] == int(np.argmin(costs))
        mine = cod[cod[:, C["region"]] == ri]
        assert int(mine[:, C["cost"]].sum()) == costs[r[4]]
        assert r[3] == np.nonzero(cod[:, C["region"]] == ri)[0][0]
    # windows of t consecutive positions
    for ri, r in enumerate(reg):
        size = pp[r[0] + 1] - pp[r[0]]
        assert r[1] % t == 0 and r[2] == min(t, size - r[1])


@pytest.mark.parametrize("seed", range(10))
def test_random_spmv_plans(seed):
    rng = np.random.default_rng(seed)
    A = I.random_csr(int(rng.integers(1, 300)), int(rng.integers(1, 300)), seed,
                     density=float(rng.uniform(0.005, 0.05)), runs=bool(seed % 2))
    check_plan(0, A, O.inspect(0, A, 64))


@pytest.mark.parametrize("seed", range(10))
def test_random_sptrsv_plans(seed):
    L = I.random_lower(int(np.random.default_rng(seed).integers(1, 250)), seed,
                       density=0.03, runs=bool(seed % 2))
    check_plan(1, L, O.inspect(1, L, 64))
    U, _ = O.transpose(L)
    check_plan(2, U, O.inspect(2, U, 64))


@pytest.mark.parametrize("t", [1, 2, 7, 64, 1024])
def test_windows(t):
    A = I.c1_laplace2d().A
    check_plan(0, A, O.inspect(0, A, t), t)


def test_stencils_and_batch_members():
    w = I.c1_laplace2d()
    check_plan(0, w.A, O.inspect(0, w.A))
    check_plan(1, w.L, O.inspect(1, w.L))
    for b in range(3):
        L = I.batch_matrix(b, n_lo=300, n_hi=900)["L"]
        check_plan(1, L, O.inspect(1, L))


def test_strided_count_monotone():
    # each flag is closed under prefixes, so k(u, m) never rises with m
    for seed in range(20):
        A = I.random_csr(40, 60, seed, density=0.05, runs=True)
        rng = np.random.default_rng(seed)
        u = int(rng.integers(0, 30))
        prev = 3
        for m in range(1, 40 - u + 1):
            fl, _ = O.classify(0, A, np.arange(u, u + m))
            k = O.flags_count(fl)
            assert k <= prev
            prev = k


def test_reverse_levels_transposed_plan():
    L = I.c1_laplace2d().L
    pT, perm = O.inspect_adjoint(1, L)
    assert pT["header"][0] == 2
    # the longest path is the same, read backwards
    assert pT["header"][5] == 127
    U, perm2 = O.transpose(L)
    assert np.array_equal(perm, perm2)
    check_plan(2, U, pT)


def test_sampled_windows_match_full():
    L = I.batch_matrix(1, n_lo=2000, n_hi=3000)["L"]
    full = O.inspect(1, L)
    samp = O.inspect(1, L, sample=5)
    for ri, r in enumerate(samp["regions"]):
        if r[4] < 0:
            continue
        assert np.array_equal(r[[0, 1, 2, 4, 5, 6, 7]], full["regions"][ri][[0, 1, 2, 4, 5, 6, 7]])
        a = samp["codelets"][samp["codelets"][:, C["region"]] == ri]
        b = full["codelets"][full["codelets"][:, C["region"]] == ri]
        keep = [i for i in range(18) if i != C["aux_off"]]
        assert np.array_equal(a[:, keep], b[:, keep])
