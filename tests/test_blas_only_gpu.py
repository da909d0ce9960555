"""The BLAS-only ablation's executor (column-slice plans: rows shared by several codelets,
partial sums combined with FP64 atomics) against the CPU oracle through the C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from tolerance import check_product, check_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_12243_amd import ddf  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rnd(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, shape)


def opts(**kw):
    return ddf.ddf_opts_default(only_blas=1, **kw)


def spmv_blas_only(A, k, seed=0, window=64):
    print(f"blas-only spmv n={A.n_rows} nnz={A.nnz} k={k} t={window}", flush=True)
    plan = ddf.ddf_inspect(0, A, opts(window=window))
    X = rnd((A.n_cols, k), seed)
    y = torch.full((A.n_rows, k), np.nan, dtype=torch.float64, device=DEV)
    ddf.ddf_spmv(plan, dev(X), y, k)
    check_product(A, X, host(y), O.spmv(A, X))
    return plan


def sptrsv_blas_only(L, k, seed=0, window=64, inplace=False):
    print(f"blas-only sptrsv n={L.n_rows} nnz={L.nnz} k={k} t={window} inplace={inplace}", flush=True)
    plan = ddf.ddf_inspect(1, L, opts(window=window))
    B = rnd((L.n_rows, k), seed)
    b = dev(B)
    x = b if inplace else torch.full_like(b, np.nan)
    ddf.ddf_sptrsv(plan, b, x, k)
    check_solve(L, B, host(x), O.sptrsv(L, B))
    # a second call reuses the accumulators: they are cleared per call
    b2 = dev(2.0 * B)
    x2 = torch.full_like(b2, np.nan)
    ddf.ddf_sptrsv(plan, b2, x2, k)
    check_solve(L, 2.0 * B, host(x2), O.sptrsv(L, 2.0 * B))
    return plan


@pytest.mark.parametrize("seed", range(6))
def test_random(seed):
    rng = np.random.default_rng(900 + seed)
    A = I.random_csr(int(rng.integers(1, 400)), int(rng.integers(1, 400)), seed,
                     density=float(rng.uniform(0.005, 0.1)), empty_frac=0.2, runs=bool(seed % 2))
    spmv_blas_only(A, int(rng.choice([1, 3])), seed, window=int(rng.choice([1, 8, 64])))
    L = I.random_lower(int(rng.integers(1, 400)), seed, density=float(rng.uniform(0.0, 0.05)),
                       runs=bool(seed % 2))
    sptrsv_blas_only(L, int(rng.choice([1, 2])), seed, window=int(rng.choice([1, 8, 64])))


def test_workloads():
    w = I.c1_laplace2d()
    spmv_blas_only(w.A, 1)
    sptrsv_blas_only(w.L, 1)
    sptrsv_blas_only(w.L, 4, inplace=True)
    w = I.c5_laplace27(nx=20, k=1)
    spmv_blas_only(w.A, 1)
    sptrsv_blas_only(w.L, 1)
    w = I.c3_chung_lu(n=30000)
    spmv_blas_only(w.A, 1)


def test_adjoints_refused():
    L = I.random_lower(50, 1, density=0.1)
    plan = ddf.ddf_inspect(1, L, opts())
    lam = torch.zeros((50, 1), dtype=torch.float64, device=DEV)
    with pytest.raises(ddf.DDFError):
        ddf.ddf_sptrsv_adjoint(plan, dev(L.values), lam, lam, lam, None, 1)
