"""Batched solve (forward and adjoint) on the GPU against the oracle per matrix, one launch per
level and one persistent dataflow launch; hipGraph replays against direct launches; per-matrix
launches of the dataflow solve give the same bits as the one-launch dataflow solve."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I
from tolerance import check_gv, check_gv_solve, check_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_12243_amd import ddf  # noqa: E402

DEV = "cuda:0"


def make_batch(nmat, n_lo, n_hi, path=0):
    mats = [I.batch_matrix(b, n_lo=n_lo, n_hi=n_hi) for b in range(nmat)]
    plan = ddf.ddf_inspect_batch(1, [m["L"] for m in mats], [m["k"] for m in mats],
                                 ddf.ddf_opts_default(solve_path=path))
    vals = np.concatenate([m["L"].values for m in mats])
    B = np.concatenate([m["B"].ravel() for m in mats])
    G = np.concatenate([m["G"].ravel() for m in mats])
    return mats, plan, vals, B, G


def split(vec, mats):
    out, o = [], 0
    for m in mats:
        n = m["L"].n_rows * m["k"]
        out.append(vec[o:o + n].reshape(m["L"].n_rows, m["k"]))
        o += n
    return out


def split_vals(vec, mats):
    out, o = [], 0
    for m in mats:
        out.append(vec[o:o + m["L"].nnz])
        o += m["L"].nnz
    return out


@pytest.mark.parametrize("path", [3, 1])  # a launch per level, one persistent launch (default)
@pytest.mark.parametrize("nmat,n_lo,n_hi", [(6, 300, 3000), (24, 1000, 20000)])
def test_batch_forward_adjoint(nmat, n_lo, n_hi, path):
    print(f"batch nmat={nmat} path={path}", flush=True)
    mats, plan, vals, B, G = make_batch(nmat, n_lo, n_hi, path)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    dv, db, dg = d(vals), d(B), d(G)
    dx = torch.full_like(db, np.nan)
    ddf.ddf_sptrsv_batch(plan, dv, db, dx)
    ddf.ddf_plan_sync_status(plan)
    X = dx.cpu().numpy()
    refs = []
    for m, x in zip(mats, split(X, mats)):
        ref = O.sptrsv(m["L"], m["B"])
        check_solve(m["L"], m["B"], x, ref)
        refs.append(ref)
    # per-matrix launches of the dataflow solve: the same bits as the one-launch dataflow solve
    # (the same lanes sum the same ops in the same order), and the oracle's values either way
    dx2 = torch.full_like(db, np.nan)
    ddf.ddf_sptrsv_batch_per_matrix(plan, dv, db, dx2)
    ddf.ddf_plan_sync_status(plan)
    if path == 1:
        assert np.array_equal(dx2.cpu().numpy(), X)
    for m, x, ref in zip(mats, split(dx2.cpu().numpy(), mats), refs):
        check_solve(m["L"], m["B"], x, ref)
    # adjoint
    dxf = d(np.concatenate([r.ravel() for r in refs]))
    dgb = torch.full_like(db, np.nan)
    dgv = torch.full_like(dv, np.nan)
    ddf.ddf_sptrsv_batch_adjoint(plan, dv, dxf, dg, dgb, dgv)
    ddf.ddf_plan_sync_status(plan)
    for m, gb, gv, ref in zip(mats, split(dgb.cpu().numpy(), mats), split_vals(dgv.cpu().numpy(), mats), refs):
        GB, GV = O.sptrsv_adj(m["L"], ref, m["G"])
        check_solve(m["L"], m["G"], gb, GB, transposed=True)
        check_gv_solve(m["L"], ref, gb, GB, gv, GV)


@pytest.mark.parametrize("path", [3, 1])
def test_graph_replays(path):
    print(f"graph replays path={path}", flush=True)
    mats, plan, vals, B, G = make_batch(8, 500, 5000, path)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    dv, db = d(vals), d(B)
    direct = torch.empty_like(db)
    ddf.ddf_sptrsv_batch(plan, dv, db, direct)
    torch.cuda.synchronize()
    ref = direct.cpu().numpy()
    out = torch.full_like(db, np.nan)
    g = ddf.ddf_graph_create_batch(plan, 0, dv, db, None, out, None)
    for rep in range(4):
        out.fill_(np.nan)  # eager work between replays
        torch.cuda.synchronize()
        ddf.ddf_graph_launch(g)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"
    ddf.ddf_plan_sync_status(plan)
    g.close()


@pytest.mark.parametrize("path", [3, 1])
def test_adjoint_graph_replays(path):
    # the batched adjoint (transposed solve and value gradient) captured once and replayed, with
    # eager work between the replays: every replay equals the direct call, which the oracle checks
    print(f"adjoint graph replays path={path}", flush=True)
    mats, plan, vals, B, G = make_batch(8, 500, 5000, path)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    refs = [O.sptrsv(m["L"], m["B"]) for m in mats]
    dv, dg, dxf = d(vals), d(G), d(np.concatenate([r.ravel() for r in refs]))
    gb, gv = torch.empty_like(dg), torch.empty_like(dv)
    ddf.ddf_sptrsv_batch_adjoint(plan, dv, dxf, dg, gb, gv)
    ddf.ddf_plan_sync_status(plan)
    want_gb, want_gv = gb.cpu().numpy().copy(), gv.cpu().numpy().copy()
    for m, lam, gvm, ref in zip(mats, split(want_gb, mats), split_vals(want_gv, mats), refs):
        GBr, GVr = O.sptrsv_adj(m["L"], ref, m["G"])
        check_solve(m["L"], m["G"], lam, GBr, transposed=True)
        check_gv_solve(m["L"], ref, lam, GBr, gvm, GVr)
    out_gb, out_gv = torch.full_like(dg, np.nan), torch.full_like(dv, np.nan)
    g = ddf.ddf_graph_create_batch(plan, 1, dv, dg, dxf, out_gb, out_gv)
    for rep in range(3):
        out_gb.fill_(np.nan)
        out_gv.fill_(np.nan)
        torch.cuda.synchronize()
        ddf.ddf_graph_launch(g)
        torch.cuda.synchronize()
        assert np.array_equal(out_gb.cpu().numpy(), want_gb), f"replay {rep}"
        assert np.array_equal(out_gv.cpu().numpy(), want_gv), f"replay {rep}"
        ddf.ddf_sptrsv_batch_adjoint(plan, dv, dxf, dg, gb, gv)  # eager work between replays
        torch.cuda.synchronize()
    ddf.ddf_plan_sync_status(plan)
    g.close()


def test_full_batch_workload():
    # all 256 matrices of the batch workload (n log-uniform in [1e3, 2e5], 1..32 right-hand
    # sides), forward and adjoint, every member against the oracle
    print("full batch workload", flush=True)
    w = I.workload("c4")
    mats = w.batch
    Ls = [m["L"] for m in mats]
    plan = ddf.ddf_inspect_batch(1, Ls, [m["k"] for m in mats])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    dv = d(np.concatenate([L.values for L in Ls]))
    db = d(np.concatenate([m["B"].ravel() for m in mats]))
    dg = d(np.concatenate([m["G"].ravel() for m in mats]))
    dx = torch.full_like(db, np.nan)
    ddf.ddf_sptrsv_batch(plan, dv, db, dx)
    ddf.ddf_plan_sync_status(plan)
    refs = [O.sptrsv(m["L"], m["B"]) for m in mats]
    for m, x, ref in zip(mats, split(dx.cpu().numpy(), mats), refs):
        check_solve(m["L"], m["B"], x, ref)
    gb, gv = torch.full_like(db, np.nan), torch.full_like(dv, np.nan)
    ddf.ddf_sptrsv_batch_adjoint(plan, dv, d(np.concatenate([r.ravel() for r in refs])), dg, gb, gv)
    ddf.ddf_plan_sync_status(plan)
    for m, lam, gvm, ref in zip(mats, split(gb.cpu().numpy(), mats), split_vals(gv.cpu().numpy(), mats), refs):
        GBr, GVr = O.sptrsv_adj(m["L"], ref, m["G"])
        check_solve(m["L"], m["G"], lam, GBr, transposed=True)
        check_gv_solve(m["L"], ref, lam, GBr, gvm, GVr)


def test_graph_refused_after_autotune():
    # tuning replaces the schedule buffers a captured graph reads: its replay is refused
    print("graph after autotune", flush=True)
    mats, plan, vals, B, G = make_batch(4, 300, 2000, 1)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    dv, db = d(vals), d(B)
    out = torch.empty_like(db)
    g = ddf.ddf_graph_create_batch(plan, 0, dv, db, None, out, None)
    ddf.ddf_graph_launch(g)
    torch.cuda.synchronize()
    ddf.ddf_autotune(plan, ddf.DDF_OP_SPTRSV, 1, budget_ms=100)
    with pytest.raises(ddf.DDFError) as e:
        ddf.ddf_graph_launch(g)
    assert e.value.status == ddf.DDF_E_ARG
    g.close()
    g2 = ddf.ddf_graph_create_batch(plan, 0, dv, db, None, out, None)
    ddf.ddf_graph_launch(g2)
    torch.cuda.synchronize()
    ddf.ddf_plan_sync_status(plan)
    for m, x in zip(mats, split(out.cpu().numpy(), mats)):
        check_solve(m["L"], m["B"], x, O.sptrsv(m["L"], m["B"]))
    g2.close()


def test_dataflow_batch_reuses_output_buffer():
    # consecutive dataflow solves with different right-hand sides into one output buffer
    mats, plan, vals, B, G = make_batch(5, 2000, 9000, path=1)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    dv, dx = d(vals), torch.full((B.size,), np.nan, dtype=torch.float64, device=DEV)
    for rep in range(3):
        Bs = B * (rep + 1) - rep
        ddf.ddf_sptrsv_batch(plan, dv, d(Bs), dx)
        ddf.ddf_plan_sync_status(plan)
        for m, x, b in zip(mats, split(dx.cpu().numpy(), mats), split(Bs, mats)):
            check_solve(m["L"], b, x, O.sptrsv(m["L"], b))
