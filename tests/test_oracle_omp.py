"""The many-core oracle loops (OpenMP over independent rows, the benchmark's many-core CPU
baseline) pinned to the serial oracle: the product and forward substitution keep each row's
serial order (bitwise equal); the adjoints sum the same terms in another order (within the
parity tolerances)."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from tolerance import check_product, check_solve


@pytest.mark.parametrize("case", ["c1", "c5", "random", "lower_small"])
def test_many_core_matches_serial(case):
    rng = np.random.default_rng(3)
    if case == "c1":
        w = I.c1_laplace2d()
        A, L, k = w.A, w.L, 1
    elif case == "c5":
        w = I.c5_laplace27(nx=14, k=8)
        A, L, k = w.A, w.L, 8
    elif case == "random":
        A = I.random_csr(700, 500, 5, density=0.02, runs=True)
        L, k = I.random_lower(5000, 6, density=0.001, runs=True), 3
    else:
        A = I.random_csr(40, 60, 7, density=0.1)
        L, k = I.random_lower(300, 8, density=0.02), 2
    X = rng.uniform(-1, 1, (A.n_cols, k))
    G = rng.uniform(-1, 1, (A.n_rows, k))
    ma = O.ManyCore(A)
    assert np.array_equal(ma.spmv(X), O.spmv(A, X))
    gx, gv = ma.spmv_adj(X, G)
    gx_ref, gv_ref = O.spmv_adj(A, X, G)
    AT, _ = O.transpose(A)
    check_product(AT, G, gx, gx_ref)
    assert np.array_equal(gv, gv_ref)
    B = rng.uniform(-1, 1, (L.n_rows, k))
    Gx = rng.uniform(-1, 1, (L.n_rows, k))
    mc = O.ManyCore(L, triangular=True)
    x_ref = O.sptrsv(L, B)
    assert np.array_equal(mc.sptrsv(B), x_ref)
    gb, gvl = mc.sptrsv_adj(x_ref, Gx)
    gb_ref, gvl_ref = O.sptrsv_adj(L, x_ref, Gx)
    check_solve(L, Gx, gb, gb_ref, transposed=True)
    assert np.allclose(gvl, gvl_ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(gvl_ref)))


def test_reverse_level_sets():
    # the reverse levels of U = L^T are the levels of the transposed solve: every row of U
    # reads only rows of earlier reverse levels, and the count equals the forward count
    L = I.random_lower(2000, 9, density=0.003)
    mc = O.ManyCore(L, triangular=True)
    rl = np.empty(L.n_rows, dtype=np.int64)
    for l in range(mc.ulptr.size - 1):
        rl[mc.ulrows[mc.ulptr[l]:mc.ulptr[l + 1]]] = l
    for i in range(L.n_rows):
        cols = mc.ciT[mc.rpT[i] + 1:mc.rpT[i + 1]]
        assert np.all(rl[cols] < rl[i])
        if cols.size:
            assert rl[i] == 1 + rl[cols].max()
    assert mc.ulptr.size == mc.lptr.size
