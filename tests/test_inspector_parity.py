"""Library inspector (C ABI, host-only plans) against the oracle inspector: canonical tables
must be bit-exact, forward and adjoint, on crafted, random and workload patterns."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import ddf
from paper_2111_12243_amd import inputs as I

KEYS = ["header", "part_ptr", "part_rows", "regions", "codelets", "aux"]


def host_plan(kind, A, t=64, threads=0, adjoint=1, only_blas=0):
    return ddf.ddf_inspect(kind, A, ddf.ddf_opts_default(host_only=1, window=t, threads=threads,
                                                         build_adjoint=adjoint, only_blas=only_blas))


def assert_same(lib_tabs, ref_tabs):
    for k in KEYS:
        assert lib_tabs[k].dtype == ref_tabs[k].dtype or k == "aux"
        assert np.array_equal(lib_tabs[k], ref_tabs[k]), k


def check(kind, A, t=64, threads=0, only_blas=False):
    p = host_plan(kind, A, t, threads, only_blas=int(only_blas))
    assert_same(ddf.ddf_plan_export(p, 0), O.inspect(kind, A, t, only_blas=only_blas))
    ref, perm = O.inspect_adjoint(kind, A, t, only_blas=only_blas)
    got = ddf.ddf_plan_export(p, 1)
    assert_same(got, ref)
    assert np.array_equal(got["perm"], perm)


def test_c1_both_kinds():
    w = I.c1_laplace2d()
    check(0, w.A)
    check(1, w.L)


@pytest.mark.parametrize("seed", range(25))
def test_random_spmv(seed):
    rng = np.random.default_rng(seed)
    A = I.random_csr(int(rng.integers(0, 300)), int(rng.integers(1, 300)), seed,
                     density=float(rng.uniform(0.002, 0.08)), empty_frac=float(rng.uniform(0, 0.5)),
                     runs=bool(seed % 2))
    check(0, A, t=int(rng.choice([1, 3, 16, 64, 100])))


@pytest.mark.parametrize("seed", range(25))
def test_random_sptrsv(seed):
    rng = np.random.default_rng(100 + seed)
    L = I.random_lower(int(rng.integers(1, 260)), seed, density=float(rng.uniform(0.0, 0.06)),
                       runs=bool(seed % 2))
    check(1, L, t=int(rng.choice([1, 2, 32, 64, 128])))


def test_crafted_shapes():
    n = 130
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.ones(n))
    check(0, eye)
    check(1, eye)
    # dense rows, single entries, one giant row
    rows = np.concatenate([np.zeros(200, int), np.arange(1, 40), np.full(3, 40)])
    cols = np.concatenate([np.arange(200), np.arange(1, 40), [0, 100, 199]])
    A = I.csr_from_pairs(41, 200, rows, cols, np.ones(rows.size))
    check(0, A, t=7)
    # empty matrix and empty rows only
    check(0, I.CSR(5, 4, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0)))


def test_threads_do_not_change_tables():
    w = I.c4_batch(1).batch[0]["L"]
    a = ddf.ddf_plan_export(host_plan(1, w, threads=1), 0)
    b = ddf.ddf_plan_export(host_plan(1, w, threads=8), 0)
    assert_same(a, b)


@pytest.mark.parametrize("b", range(6))
def test_batch_members(b):
    m = I.batch_matrix(b, n_lo=500, n_hi=20000)
    check(1, m["L"])


def test_c2_scaled():
    w = I.c2_stencil27_offband(nx=24)
    check(0, w.A)
    check(1, w.L)


def test_c3_scaled():
    w = I.c3_chung_lu(n=60000)
    check(0, w.A)


def test_c5_scaled():
    w = I.c5_laplace27(nx=30, k=1)
    check(0, w.A)
    check(1, w.L)


# BLAS-only ablation (every window covered by column slices): same bar, forward and adjoint.
@pytest.mark.parametrize("seed", range(12))
def test_blas_only_random(seed):
    rng = np.random.default_rng(300 + seed)
    A = I.random_csr(int(rng.integers(0, 200)), int(rng.integers(1, 200)), seed,
                     density=float(rng.uniform(0.002, 0.1)), empty_frac=float(rng.uniform(0, 0.4)),
                     runs=bool(seed % 2))
    check(0, A, t=int(rng.choice([1, 4, 64])), only_blas=True)
    L = I.random_lower(int(rng.integers(1, 200)), seed, density=float(rng.uniform(0.0, 0.08)),
                       runs=bool(seed % 2))
    check(1, L, t=int(rng.choice([1, 8, 64])), only_blas=True)


def test_blas_only_workloads():
    w = I.c1_laplace2d()
    check(0, w.A, only_blas=True)
    check(1, w.L, only_blas=True)
    w = I.c5_laplace27(nx=14, k=1)
    check(0, w.A, threads=4, only_blas=True)
    check(1, w.L, threads=4, only_blas=True)
