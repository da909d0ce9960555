"""The no-allocation transposed solve (ddf_sptrsv_adjoint_noalloc: scratch in the library's
static device array) against ddf_sptrsv_adjoint on the same plan: two calls in a row, the
second on a smaller matrix, each with the parity measures of the oracle comparison."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from tolerance import check_gv_solve, check_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_12243_amd import ddf  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


@pytest.mark.gpu
def test_noalloc_matches_allocating_entry_point():
    cases = [(I.c5_laplace27(nx=40, k=8).L, 8, 0), (I.random_lower(3000, 21, density=0.004, runs=True), 3, 1)]
    for L, k, seed in cases:
        print(f"no-alloc transposed solve n={L.n_rows} nnz={L.nnz} k={k}", flush=True)
        plan = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=1))
        rng = np.random.default_rng(seed)
        B, G = rng.uniform(-1, 1, (L.n_rows, k)), rng.uniform(-1, 1, (L.n_rows, k))
        xref = O.sptrsv(L, B)
        GB, GV = O.sptrsv_adj(L, xref, G)
        vals, x, g = dev(L.values), dev(xref), dev(G)
        gb1, gv1 = torch.full_like(g, np.nan), torch.full((L.nnz,), np.nan, dtype=torch.float64, device=DEV)
        ddf.ddf_sptrsv_adjoint(plan, vals, x, g, gb1, gv1, k)
        gb2, gv2 = torch.full_like(g, np.nan), torch.full((L.nnz,), np.nan, dtype=torch.float64, device=DEV)
        ddf.ddf_sptrsv_adjoint_noalloc(plan, vals, x, g, gb2, gv2, k)
        ddf.ddf_plan_sync_status(plan)
        a, b = gb2.cpu().numpy(), gv2.cpu().numpy()
        check_solve(L, G, a, GB, transposed=True)
        check_gv_solve(L, xref, a, GB, b, GV)
        # the same kernels on the same values: the same bits as the allocating entry point
        assert np.array_equal(a, gb1.cpu().numpy())
        assert np.array_equal(b, gv1.cpu().numpy())
        # in place (gb == gx): one launch per level, values gathered into the static scratch
        gi = dev(G)
        ddf.ddf_sptrsv_adjoint_noalloc(plan, vals, x, gi, gi, None, k)
        ddf.ddf_plan_sync_status(plan)
        check_solve(L, G, gi.cpu().numpy(), GB, transposed=True)


@pytest.mark.gpu
def test_noalloc_rejects_oversized_plans():
    # more stored values than the static scratch holds: DDF_E_ARG before any launch
    n = 2100000
    rows = np.concatenate([np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(n - 1), np.arange(n)])
    L = I.csr_from_pairs(n, n, rows, cols, np.full(rows.size, 2.0))
    assert L.nnz > (1 << 22)
    plan = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=1))
    g = torch.ones((n, 1), dtype=torch.float64, device=DEV)
    out = torch.full_like(g, 7.0)
    with pytest.raises(ddf.DDFError) as e:
        ddf.ddf_sptrsv_adjoint_noalloc(plan, None, None, g, out, None, 1)
    assert e.value.status == ddf.DDF_E_ARG and "static scratch" in str(e.value)
    assert (out.cpu().numpy() == 7.0).all()
