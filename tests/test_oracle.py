"""The CPU oracle's values pinned to things other than itself: dense brute force, library
triangular solves, closed forms, linearity, residuals and finite differences."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from paper_2111_12243_amd import inputs as I


def lap1d(n):
    rows, cols, vals = [], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                rows.append(i), cols.append(j), vals.append(v)
    return I.csr_from_pairs(n, n, np.array(rows), np.array(cols), np.array(vals))


def lap2d(N):
    return I.laplacian(N, N, 1, I.OFFS_5PT, 4.0)


# ---------------------------------------------------------------- SpMV (O1)

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("k", [1, 3])
def test_spmv_dense_bruteforce(seed, k):
    rng = np.random.default_rng(seed)
    nr, nc = int(rng.integers(1, 64)), int(rng.integers(1, 64))
    A = I.random_csr(nr, nc, seed, density=0.3, runs=bool(seed % 2))
    X = rng.uniform(-1, 1, (nc, k))
    Y = O.spmv(A, X)
    ref = A.to_dense() @ X
    assert np.allclose(Y, ref, rtol=1e-14, atol=1e-14)


def test_spmv_identity_and_diagonal():
    n = 50
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.ones(n))
    X = np.random.default_rng(1).uniform(-1, 1, (n, 2))
    assert np.array_equal(O.spmv(eye, X), X)
    d = np.random.default_rng(2).uniform(0.5, 2, n)
    D = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), d)
    assert np.array_equal(O.spmv(D, X), d[:, None] * X)


def test_spmv_lap1d_closed_forms():
    n = 37
    A = lap1d(n)
    y = O.spmv(A, np.ones((n, 1)))[:, 0]
    e = np.zeros(n)
    e[0] = e[-1] = 1
    assert np.array_equal(y, e)
    y = O.spmv(A, np.arange(n, dtype=float)[:, None])[:, 0]
    e = np.zeros(n)
    e[0], e[-1] = -1.0, float(n)
    assert np.array_equal(y, e)
    x = np.sin(np.pi * (np.arange(n) + 1) / (n + 1))
    lam = 2 * (1 - np.cos(np.pi / (n + 1)))
    y = O.spmv(A, x[:, None])[:, 0]
    assert np.max(np.abs(y - lam * x)) < 1e-14


def test_spmv_lap2d_closed_forms():
    N = 12
    A = lap2d(N)
    y = O.spmv(A, np.ones((N * N, 1)))[:, 0].reshape(N, N)
    missing = np.zeros((N, N))
    missing[0, :] += 1
    missing[-1, :] += 1
    missing[:, 0] += 1
    missing[:, -1] += 1
    assert np.array_equal(y, missing)
    ii = np.tile(np.arange(N, dtype=float), N)  # x = i^2, i the fast index
    y = O.spmv(A, (ii ** 2)[:, None])[:, 0].reshape(N, N)
    assert np.array_equal(y[1:-1, 1:-1], np.full((N - 2, N - 2), -2.0))
    for p, q in ((1, 1), (2, 5), (N, 3)):
        s1 = np.sin(p * np.pi * (np.arange(N) + 1) / (N + 1))
        s2 = np.sin(q * np.pi * (np.arange(N) + 1) / (N + 1))
        x = np.outer(s2, s1).ravel()  # rows j (slow) x cols i (fast)
        lam = 4 - 2 * np.cos(p * np.pi / (N + 1)) - 2 * np.cos(q * np.pi / (N + 1))
        y = O.spmv(A, x[:, None])[:, 0]
        assert np.max(np.abs(y - lam * x)) < 1e-13


def test_spmv_linearity():
    A = I.random_csr(40, 30, 7, density=0.2)
    rng = np.random.default_rng(3)
    x, z = rng.uniform(-1, 1, (30, 2)), rng.uniform(-1, 1, (30, 2))
    a, b = 0.75, -1.25
    lhs = O.spmv(A, a * x + b * z)
    rhs = a * O.spmv(A, x) + b * O.spmv(A, z)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_spmv_empty():
    A = I.CSR(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert O.spmv(A, np.ones((5, 1))).shape == (0, 1)
    A = I.CSR(3, 4, np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(O.spmv(A, np.ones((4, 2))), np.zeros((3, 2)))


# ---------------------------------------------------------------- SpTRSV (O2)

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("k", [1, 4])
def test_sptrsv_library_solve(seed, k):
    n = int(np.random.default_rng(seed).integers(1, 64))
    L = I.random_lower(n, seed, density=0.3, runs=bool(seed % 2))
    B = np.random.default_rng(seed + 100).uniform(-1, 1, (n, k))
    X = O.sptrsv(L, B)
    ref = sl.solve_triangular(L.to_dense(), B, lower=True)
    assert np.max(np.abs(X - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    # residual ||B - L X|| relative to |L||X| + |B|
    Ld = L.to_dense()
    res = np.max(np.abs(B - Ld @ X))
    scale = np.max(np.abs(Ld) @ np.abs(X)) + np.max(np.abs(B))
    assert res <= 1e-15 * scale * n


def test_sptrsv_closed_forms():
    n = 40
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.ones(n))
    B = np.random.default_rng(0).uniform(-1, 1, (n, 3))
    assert np.array_equal(O.sptrsv(eye, B), B)
    d = np.random.default_rng(1).uniform(0.5, 2, n)
    D = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), d)
    assert np.array_equal(O.sptrsv(D, B), B / d[:, None])
    # bidiagonal (a on the diagonal, c below): b = e0 gives x_i = (1/a)(-c/a)^i
    a, c = 2.0, 0.5
    rows = np.concatenate([np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(n - 1), np.arange(n)])
    vals = np.concatenate([np.full(n - 1, c), np.full(n, a)])
    Lb = I.csr_from_pairs(n, n, rows, cols, vals)
    b = np.zeros((n, 1))
    b[0] = 1
    x = O.sptrsv(Lb, b)[:, 0]
    assert np.array_equal(x, (1 / a) * (-c / a) ** np.arange(n))
    # lower part of the 1D Laplacian with b = 1: x_i = 1 - 2^-(i+1), exact in binary64
    Ll = I.tril(lap1d(n))
    x = O.sptrsv(Ll, np.ones((n, 1)))[:, 0]
    assert np.array_equal(x, 1 - 2.0 ** -(np.arange(n) + 1))


def test_sptrsv_in_place():
    L = I.random_lower(30, 5)
    B = np.random.default_rng(5).uniform(-1, 1, (30, 2))
    X = O.sptrsv(L, B)
    rp, ci, v = (np.ascontiguousarray(a) for a in (L.row_ptr, L.col_idx, L.values))
    buf = B.copy()
    O.lib().orc_sptrsv(30, O._p(rp), O._p(ci), O._p(v), 2, O._p(buf), O._p(buf))
    assert np.array_equal(buf, X)


# ---------------------------------------------------------------- adjoints (O3, O4)

@pytest.mark.parametrize("seed", range(4))
def test_spmv_adjoint_dense(seed):
    rng = np.random.default_rng(seed)
    A = I.random_csr(33, 27, seed, density=0.25)
    k = 3
    X, G = rng.uniform(-1, 1, (27, k)), rng.uniform(-1, 1, (33, k))
    GX, GV = O.spmv_adj(A, X, G)
    assert np.allclose(GX, A.to_dense().T @ G, rtol=1e-14, atol=1e-14)
    rows = np.repeat(np.arange(33), np.diff(A.row_ptr))
    assert np.allclose(GV, (G @ X.T)[rows, A.col_idx], rtol=1e-14, atol=1e-14)


def test_spmv_adjoint_finite_differences():
    # loss = <G, A X> is linear in X and in the values: central differences are exact up to
    # rounding
    rng = np.random.default_rng(9)
    A = I.random_csr(12, 10, 9, density=0.4)
    X, G = rng.uniform(-1, 1, (10, 2)), rng.uniform(-1, 1, (12, 2))
    GX, GV = O.spmv_adj(A, X, G)
    loss = lambda A_, X_: float(np.sum(G * O.spmv(A_, X_)))
    h = 0.5
    for j in range(10):
        for r in range(2):
            Xp, Xm = X.copy(), X.copy()
            Xp[j, r] += h
            Xm[j, r] -= h
            assert abs((loss(A, Xp) - loss(A, Xm)) / (2 * h) - GX[j, r]) < 1e-13
    for e in range(A.nnz):
        Ap = I.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.values.copy())
        Am = I.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.values.copy())
        Ap.values[e] += h
        Am.values[e] -= h
        assert abs((loss(Ap, X) - loss(Am, X)) / (2 * h) - GV[e]) < 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_sptrsv_adjoint_library(seed):
    rng = np.random.default_rng(seed)
    n, k = 35, 3
    L = I.random_lower(n, seed + 50, density=0.25)
    B, G = rng.uniform(-1, 1, (n, k)), rng.uniform(-1, 1, (n, k))
    X = O.sptrsv(L, B)
    GB, GV = O.sptrsv_adj(L, X, G)
    Ld = L.to_dense()
    lam = sl.solve_triangular(Ld, G, lower=True, trans="T")
    assert np.max(np.abs(GB - lam)) <= 1e-13 * max(1, np.max(np.abs(lam)))
    rows = np.repeat(np.arange(n), np.diff(L.row_ptr))
    ref = -(lam @ X.T)[rows, L.col_idx]
    assert np.max(np.abs(GV - ref)) <= 1e-13 * max(1, np.max(np.abs(ref)))


def test_sptrsv_adjoint_diagonal_closed_form():
    n = 20
    rng = np.random.default_rng(4)
    d = rng.uniform(0.5, 2, n)
    D = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), d)
    b, g = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    x = O.sptrsv(D, b)
    GB, GV = O.sptrsv_adj(D, x, g)
    assert np.array_equal(GB[:, 0], g[:, 0] / d)
    assert np.allclose(GV, -g[:, 0] * b[:, 0] / d ** 2, rtol=1e-15, atol=0)


def test_sptrsv_adjoint_finite_differences():
    rng = np.random.default_rng(11)
    n = 9
    L = I.random_lower(n, 11, density=0.5)
    B, G = rng.uniform(-1, 1, (n, 2)), rng.uniform(-1, 1, (n, 2))
    X = O.sptrsv(L, B)
    GB, GV = O.sptrsv_adj(L, X, G)
    loss = lambda L_, B_: float(np.sum(G * O.sptrsv(L_, B_)))
    h = 1e-6
    for j in range(n):
        Bp, Bm = B.copy(), B.copy()
        Bp[j, 0] += h
        Bm[j, 0] -= h
        assert abs((loss(L, Bp) - loss(L, Bm)) / (2 * h) - GB[j, 0]) < 1e-8
    for e in range(L.nnz):
        Lp = I.CSR(n, n, L.row_ptr, L.col_idx, L.values.copy())
        Lm = I.CSR(n, n, L.row_ptr, L.col_idx, L.values.copy())
        Lp.values[e] += h
        Lm.values[e] -= h
        assert abs((loss(Lp, B) - loss(Lm, B)) / (2 * h) - GV[e]) < 1e-7


# ---------------------------------------------------------------- transpose / validation

def test_transpose_dense_and_perm():
    A = I.random_csr(23, 31, 3, density=0.2)
    AT, perm = O.transpose(A)
    assert np.array_equal(I.CSR(AT.n_rows, AT.n_cols, AT.row_ptr, AT.col_idx,
                                AT.values).to_dense(), A.to_dense().T)
    assert np.array_equal(AT.values, A.values[perm])
    # stable: within a row of A^T, source rows ascend
    for j in range(AT.n_rows):
        seg = perm[AT.row_ptr[j]:AT.row_ptr[j + 1]]
        assert np.all(np.diff(seg) > 0)


def test_validate_rejects():
    good = I.random_lower(10, 1)
    assert O.validate(1, good) == 0
    assert O.validate(0, good) == 0
    bad = I.CSR(10, 10, good.row_ptr.copy(), good.col_idx.copy(), good.values)
    bad.row_ptr[3], bad.row_ptr[4] = bad.row_ptr[4], bad.row_ptr[3]
    assert O.validate(0, bad) != 0
    bad = I.CSR(10, 10, good.row_ptr, good.col_idx.copy(), good.values)
    bad.col_idx[-1] = 10
    assert O.validate(0, bad) == 3
    A = I.random_csr(10, 10, 2, density=0.5)
    assert O.validate(1, A) == 6  # not lower with diagonal last
    U, _ = O.transpose(good)
    assert O.validate(2, U) == 0 and O.validate(1, U) == 6
