"""Schedules picked by the autotuner, run under the parity measures: every executor op tuned on
scaled workloads and a batch, then checked against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from tolerance import check_gv, check_gv_solve, check_product, check_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_12243_amd import ddf  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


@pytest.mark.parametrize("name,kw", [("c2", dict(nx=24)), ("c3", dict(n=100000)), ("c5", dict(nx=24, k=8))])
def test_tuned_single(name, kw):
    print(f"autotune {name} {kw}", flush=True)
    w = I.workload(name, **kw)
    A, L, k = w.A, w.L, w.k
    pA = ddf.ddf_inspect(0, A)
    ddf.ddf_autotune(pA, ddf.DDF_OP_SPMV, k, budget_ms=400)
    ddf.ddf_autotune(pA, ddf.DDF_OP_SPMV_ADJ, k, budget_ms=400)
    print("  SpMV schedule", {key: ddf.ddf_plan_info(pA)[key] for key in ("ops_per_lane", "rows_passes", "xcd_remap")},
          flush=True)
    x, g = dev(w.X), dev(w.Gy)
    y = torch.full((A.n_rows, k), np.nan, dtype=torch.float64, device=DEV)
    ddf.ddf_spmv(pA, x, y, k)
    check_product(A, w.X, y.cpu().numpy(), O.spmv(A, w.X))
    gx = torch.full((A.n_cols, k), np.nan, dtype=torch.float64, device=DEV)
    gv = torch.full((A.nnz,), np.nan, dtype=torch.float64, device=DEV)
    ddf.ddf_spmv_adjoint(pA, dev(A.values), x, g, gx, gv, k)
    GX, GV = O.spmv_adj(A, w.X, w.Gy)
    AT, _ = O.transpose(A)
    check_product(AT, w.Gy, gx.cpu().numpy(), GX)
    check_gv(A, w.X, w.Gy, gv.cpu().numpy(), GV)
    if L is None:
        return
    pL = ddf.ddf_inspect(1, L)
    ddf.ddf_autotune(pL, ddf.DDF_OP_SPTRSV, k, budget_ms=600)
    ddf.ddf_autotune(pL, ddf.DDF_OP_SPTRSV_ADJ, k, budget_ms=600)
    info = ddf.ddf_plan_info(pL)
    print("  solve paths", info["solve_path"], info["solve_path_adj"], flush=True)
    b = dev(w.B)
    xs = torch.full_like(b, np.nan)
    ddf.ddf_sptrsv(pL, b, xs, k)
    ddf.ddf_plan_sync_status(pL)
    xref = O.sptrsv(L, w.B)
    check_solve(L, w.B, xs.cpu().numpy(), xref)
    gb = torch.full_like(b, np.nan)
    gvl = torch.full((L.nnz,), np.nan, dtype=torch.float64, device=DEV)
    ddf.ddf_sptrsv_adjoint(pL, dev(L.values), dev(xref), dev(w.Gx), gb, gvl, k)
    ddf.ddf_plan_sync_status(pL)
    GB, GVL = O.sptrsv_adj(L, xref, w.Gx)
    check_solve(L, w.Gx, gb.cpu().numpy(), GB, transposed=True)
    check_gv_solve(L, xref, gb.cpu().numpy(), GB, gvl.cpu().numpy(), GVL)


def test_tuned_batch():
    print("autotune batch", flush=True)
    mats = [I.batch_matrix(b, n_lo=500, n_hi=8000) for b in range(10)]
    Ls = [m["L"] for m in mats]
    plan = ddf.ddf_inspect_batch(1, Ls, [m["k"] for m in mats])
    ddf.ddf_autotune(plan, ddf.DDF_OP_SPTRSV, 1, budget_ms=600)
    ddf.ddf_autotune(plan, ddf.DDF_OP_SPTRSV_ADJ, 1, budget_ms=600)
    info = ddf.ddf_plan_info(plan)
    print("  batch solve paths", info["solve_path"], info["solve_path_adj"], flush=True)
    vals = dev(np.concatenate([L.values for L in Ls]))
    B = dev(np.concatenate([m["B"].ravel() for m in mats]))
    X = torch.full_like(B, np.nan)
    ddf.ddf_sptrsv_batch(plan, vals, B, X)
    ddf.ddf_plan_sync_status(plan)
    xh, off, refs = X.cpu().numpy(), 0, []
    for m in mats:
        n, k = m["L"].n_rows, m["k"]
        ref = O.sptrsv(m["L"], m["B"])
        check_solve(m["L"], m["B"], xh[off:off + n * k].reshape(n, k), ref)
        refs.append(ref)
        off += n * k
    G = dev(np.concatenate([m["G"].ravel() for m in mats]))
    GB, GV = torch.full_like(B, np.nan), torch.full_like(vals, np.nan)
    ddf.ddf_sptrsv_batch_adjoint(plan, vals, dev(np.concatenate([r.ravel() for r in refs])), G, GB, GV)
    ddf.ddf_plan_sync_status(plan)
    gbh, gvh, off, voff = GB.cpu().numpy(), GV.cpu().numpy(), 0, 0
    for m, ref in zip(mats, refs):
        n, k, nz = m["L"].n_rows, m["k"], m["L"].nnz
        GBr, GVr = O.sptrsv_adj(m["L"], ref, m["G"])
        lam = gbh[off:off + n * k].reshape(n, k)
        check_solve(m["L"], m["G"], lam, GBr, transposed=True)
        check_gv_solve(m["L"], ref, lam, GBr, gvh[voff:voff + nz], GVr)
        off += n * k
        voff += nz
