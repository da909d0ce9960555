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
