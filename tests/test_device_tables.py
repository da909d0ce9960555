"""Device tables and schedules of host-only plans, replayed on the CPU with the kernels'
indexing (tests/device_emulator.py): bounds, exact cover, dependency order, and values
against the oracle."""
import numpy as np
import pytest

import device_emulator as E
import oracle as O
from paper_2111_12243_amd import ddf
from paper_2111_12243_amd import inputs as I
from tolerance import check_gv_solve, check_product, check_solve


def hplan(kind, A, **kw):
    return ddf.ddf_inspect(kind, A, ddf.ddf_opts_default(host_only=1, **kw))


def replay_spmv(A, k=2, seed=0, **kw):
    p = hplan(0, A, **kw)
    rng = np.random.default_rng(seed)
    X, G = rng.uniform(-1, 1, (A.n_cols, k)), rng.uniform(-1, 1, (A.n_rows, k))
    F = ddf.ddf_plan_device_tables(p, 0)
    T = ddf.ddf_plan_device_tables(p, 1)
    AT, perm = O.transpose(A)
    GXr, _ = O.spmv_adj(A, X, G)
    for many in (False, True):
        check_product(A, X, E.spmv(F, A, X, many=many), O.spmv(A, X))
        gx = E.spmv(T, AT, G, vals=A.values, perm=perm, many=many)
        check_product(AT, G, gx, GXr)
    return F


def replay_solve(L, k=2, seed=0, **kw):
    p = hplan(1, L, **kw)
    rng = np.random.default_rng(seed)
    B, G = rng.uniform(-1, 1, (L.n_rows, k)), rng.uniform(-1, 1, (L.n_rows, k))
    F = ddf.ddf_plan_device_tables(p, 0)
    X = E.solve(F, L, B)
    ref = O.sptrsv(L, B)
    check_solve(L, B, X, ref)
    T = ddf.ddf_plan_device_tables(p, 1)
    U, perm = O.transpose(L)
    # the dataflow lists: forward and transposed solves in dependence order
    check_solve(L, B, E.df_solve(F, L, B), ref)
    check_solve(L, G, E.df_solve(T, U, G, kind=2, vals=L.values, perm=perm), O.sptrsv_adj(L, ref, G)[0],
                transposed=True)
    if F["thin_rec"].shape[0]:
        check_solve(L, B[:, :1], E.thin_solve(F, L, B[:, :1]), ref[:, :1])
    if T["thin_rec"].shape[0]:
        G, ref = G[:, :1], ref[:, :1]
        lam_t, gv_t = E.thin_solve(T, U, G, vals=L.values, Xf=ref)
        GBt, GVt = O.sptrsv_adj(L, ref, G)
        check_solve(L, G, lam_t, GBt, transposed=True)
        check_gv_solve(L, ref, lam_t, GBt, gv_t, GVt)
    lam = E.solve(T, U, G, kind=2, vals=L.values, perm=perm)
    check_solve(L, G, lam, O.sptrsv_adj(L, ref, G)[0], transposed=True)
    # every task of the one-launch-per-level lists solves rows (the value gradient runs over
    # the CSR pattern)
    assert not ((T["tasks"][:, 3] >> 8) & 1).any()
    return F


@pytest.mark.parametrize("seed", range(12))
def test_random_spmv_tables(seed):
    rng = np.random.default_rng(seed)
    A = I.random_csr(int(rng.integers(1, 200)), int(rng.integers(1, 200)), seed,
                     density=float(rng.uniform(0.005, 0.1)), empty_frac=float(rng.uniform(0, 0.4)),
                     runs=bool(seed % 2))
    replay_spmv(A, k=1 + seed % 3, seed=seed, ops_per_lane=int(rng.choice([1, 4, 16])),
                rows_passes=int(rng.choice([1, 2, 4])), window=int(rng.choice([8, 64])))


@pytest.mark.parametrize("seed", range(12))
def test_random_solve_tables(seed):
    rng = np.random.default_rng(70 + seed)
    L = I.random_lower(int(rng.integers(1, 160)), seed, density=float(rng.uniform(0, 0.06)), runs=bool(seed % 2))
    replay_solve(L, k=1 + seed % 3, seed=seed, ops_per_lane=int(rng.choice([1, 4, 16])),
                 rows_passes=int(rng.choice([1, 2])), window=int(rng.choice([4, 64])))


def test_workload_tables():
    w = I.c1_laplace2d()
    replay_spmv(w.A, k=1)
    F = replay_solve(w.L, k=1)
    assert F["n_counters"] == 127  # one counter per level
    w = I.c2_stencil27_offband(nx=12)
    replay_spmv(w.A, k=1)
    replay_solve(w.L, k=1)
    w = I.c5_laplace27(nx=10, k=2)
    replay_spmv(w.A, k=2)
    replay_solve(w.L, k=2)


def test_counter_protocol_2d_laplacian():
    # wide middle levels: many tasks per level, each waiting on the previous level's counter
    L = I.tril(I.laplacian(300, 300, 1, I.OFFS_5PT, 4.0))
    p = hplan(1, L, ops_per_lane=1, rows_passes=1)
    F = ddf.ddf_plan_device_tables(p, 0)
    assert F["n_counters"] == 599
    X = E.solve(F, L, np.ones((L.n_rows, 1)))
    check_solve(L, np.ones((L.n_rows, 1)), X, O.sptrsv(L, np.ones((L.n_rows, 1))))


def test_batch_schedule_per_matrix():
    mats = [I.batch_matrix(b, n_lo=200, n_hi=3000) for b in range(5)]
    Ls = [m["L"] for m in mats]
    p = ddf.ddf_inspect_batch(1, Ls, [m["k"] for m in mats], ddf.ddf_opts_default(host_only=1))
    F = ddf.ddf_plan_device_tables(p, 0)
    T = ddf.ddf_plan_device_tables(p, 1)
    PM = ddf.ddf_plan_device_tables(p, 2)
    for b, m in enumerate(mats):
        L, k = m["L"], m["k"]
        B = m["B"]
        X = E.solve(F, L, B, only_mat=b)
        ref = O.sptrsv(L, B)
        check_solve(L, B, X, ref)
        # the dataflow lists, batch (all matrices level by level) and per matrix, each in
        # dependence order
        check_solve(L, B, E.df_solve(F, L, B, only_mat=b), ref)
        check_solve(L, B, E.df_solve(PM, L, B, only_mat=b), ref)
        U, perm = O.transpose(L)
        lam = E.solve(T, U, m["G"], kind=2, vals=L.values, perm=perm, only_mat=b)
        GBr = O.sptrsv_adj(L, ref, m["G"])[0]
        check_solve(L, m["G"], lam, GBr, transposed=True)
        check_solve(L, m["G"], E.df_solve(T, U, m["G"], kind=2, vals=L.values, perm=perm, only_mat=b), GBr,
                    transposed=True)


def test_stream_tasks_single_entry_rows():
    # rows of one entry (nn = 1) and the paper's worked example, transposed
    rows = np.repeat(np.arange(3), 3)
    A = I.csr_from_pairs(3, 8, rows, np.array([0, 2, 5, 1, 3, 6, 2, 4, 7]), np.arange(1.0, 10.0))
    replay_spmv(A, k=1)
    n = 100
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.arange(1.0, n + 1))
    replay_spmv(eye, k=1)


@pytest.mark.parametrize("window", [128, 1024])
def test_stream_tasks_wide_windows(window):
    # rectangular codelets of one to three entries per row over windows wider than a wave:
    # every stream task must stay within the 64 rows one wave sums
    n = 2000
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.arange(1.0, n + 1))
    F = replay_spmv(eye, k=1, window=window)
    T = I.laplacian(n, 1, 1, [(-1, 0, 0), (0, 0, 0), (1, 0, 0)], 2.0)  # tridiagonal
    F2 = replay_spmv(T, k=1, window=window)
    for tabs in (F, F2):
        st = tabs["tasks"][(tabs["tasks"][:, 3] & E.TASK_STREAM) != 0]
        assert len(st) and (st[:, 2] - st[:, 1]).max() <= 64


def test_thin_records_workloads():
    w = I.c1_laplace2d()
    F = ddf.ddf_plan_device_tables(hplan(1, w.L), 0)
    lv = F["thin_lvl"]
    assert (lv[:, 1] > 0).sum() == 127 and lv.shape[0] == 132
    w = I.c2_stencil27_offband(nx=16)
    p = hplan(1, w.L)
    F, T = ddf.ddf_plan_device_tables(p, 0), ddf.ddf_plan_device_tables(p, 1)
    assert F["thin_rec"].shape[0] and T["thin_rec"].shape[0]
    replay_solve(w.L, k=1)
    # about 1% of rows longer than G lanes hold: they take 2G lanes
    L = I.mixed_lower(3000, 5)
    F = replay_solve(L, k=1)
    assert (F["thin_rec"][:, 19] == 1).any() and F["thin_lg"] == 0
    # a level wider than one pass is not eligible
    L = I.tril(I.laplacian(1200, 1200, 1, I.OFFS_5PT, 4.0))
    assert ddf.ddf_plan_device_tables(hplan(1, L, build_adjoint=0), 0)["thin_rec"].shape[0] == 0


def test_thin_small_ring_global_operands():
    # a 256-row ring forces most operands through the global gather path
    w = I.c2_stencil27_offband(nx=16)
    p = hplan(1, w.L, thin_ring=256)
    F, T = ddf.ddf_plan_device_tables(p, 0), ddf.ddf_plan_device_tables(p, 1)
    for D in (F, T):
        assert D["thin_ring_size"] == 256 and D["thin_rec"].shape[0]
        codes = D["thin_rec"][:, 14:19]
        assert (codes >= 0).any() and (codes[codes != E.THIN_UNUSED] < 0).any() and D["thin_ngs"] >= 1
    replay_solve(w.L, k=1, thin_ring=256)
    with pytest.raises(ddf.DDFError):
        hplan(1, w.L, thin_ring=300)



def test_thin_pinned_operands():
    # hub rows read ~30 rows far behind a 256-row ring: past two global slots per lane their
    # operands come from pinned LDS entries, written once by the rows that own them
    L = I.hub_lower(3000, 5)
    F = replay_solve(L, k=1, thin_ring=256)
    M = F["thin_ring_size"]
    codes = F["thin_rec"][:, 14:19]
    pinned = (codes <= -(M + 3)) & (codes != E.THIN_UNUSED)
    assert pinned.sum() > 50 and F["thin_ngs"] <= 2
    writers = F["thin_rec"][:, 20]
    assert (writers >= M + 2).sum() == len(set((-codes[pinned] - 1).tolist()))


def test_thin_pinned_entries_overflow():
    # hubs every third row need more than the 2048 pinned entries: the plan falls back to more
    # global slots per lane and pins nothing
    L = I.hub_lower(12000, 9, hub_every=3, hub_ops=30)
    F = replay_solve(L, k=1, thin_ring=256)
    M = F["thin_ring_size"]
    codes = F["thin_rec"][:, 14:19]
    assert F["thin_rec"].shape[0] and F["thin_ngs"] > 2
    assert not ((codes <= -(M + 3)) & (codes != E.THIN_UNUSED)).any()
    assert (F["thin_rec"][:, 20] < M).all()


def test_thin_lane_cap_sub_levels():
    # a lane cap cuts wide levels into consecutive sub-levels; the solve order stays valid
    L = I.tril(I.laplacian(150, 150, 1, I.OFFS_5PT, 4.0))
    full = ddf.ddf_plan_device_tables(hplan(1, L, thin_lanes=1024), 0)
    F = replay_solve(L, k=1, thin_lanes=64)
    used, used_full = F["thin_lvl"][:, 1], full["thin_lvl"][:, 1]
    assert used_full.max() > 128 and used.max() <= 64 and (used > 0).sum() > (used_full > 0).sum()
    assert used.sum() == used_full.sum() and F["thin_block"] == 64
    # a level wider than 1024 lanes becomes eligible once cut
    offs7 = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    L = I.tril(I.laplacian(40, 40, 40, offs7, 6.0))
    assert ddf.ddf_plan_device_tables(hplan(1, L, build_adjoint=0), 0)["thin_rec"].shape[0] == 0
    F = replay_solve(L, k=1, thin_lanes=1024)
    assert F["thin_rec"].shape[0] and F["thin_lvl"][:, 1].max() <= 1024
    with pytest.raises(ddf.DDFError):
        hplan(1, L, thin_lanes=100)


@pytest.mark.parametrize("window", [4, 64])
def test_long_row_tasks(window):
    L = I.long_rows_lower()
    F = replay_solve(L, k=3, window=window)
    p = hplan(1, L, window=window)
    T = ddf.ddf_plan_device_tables(p, 1)
    for tabs in (F, T):
        lng = (tabs["df_tasks"][:, 3] & E.DF_LONG) != 0
        assert lng.sum() >= 1 and tabs["df_lcols"].size > 0 and tabs["df_group"] == E.DF_PASS_MAX
        assert (np.flatnonzero(lng) % E.DF_PASS_MAX == 0).all()


def test_long_row_tasks_batch():
    mats = [I.batch_matrix(b, n_lo=4000, n_hi=8000) for b in (2, 5, 0)]
    Ls = [m["L"] for m in mats]
    p = ddf.ddf_inspect_batch(1, Ls, [m["k"] for m in mats], ddf.ddf_opts_default(host_only=1))
    F, T, PM = (ddf.ddf_plan_device_tables(p, w) for w in (0, 1, 2))
    assert ((F["df_tasks"][:, 3] & E.DF_LONG) != 0).any() and F["df_group"] == 1
    assert (F["df_tasks"][:, 3] == E.DF_MIXED).any() and F["df_slots"].shape[1] == 2
    for b, m in enumerate(mats):
        L, B = m["L"], m["B"]
        ref = O.sptrsv(L, B)
        check_solve(L, B, E.df_solve(F, L, B, only_mat=b), ref)
        check_solve(L, B, E.df_solve(PM, L, B, only_mat=b), ref)
        U, perm = O.transpose(L)
        check_solve(L, m["G"], E.df_solve(T, U, m["G"], kind=2, vals=L.values, perm=perm, only_mat=b),
                    O.sptrsv_adj(L, ref, m["G"])[0], transposed=True)


@pytest.mark.parametrize("seed", range(4))
def test_wide_row_tasks_dense_rows(seed):
    # rows of 17..100 ops: wide-row tasks of several rows (rows that fit 64 / R lanes)
    L = I.random_lower(160, 40 + seed, density=0.25 + 0.1 * seed)
    F = replay_solve(L, k=1 + seed, seed=seed, window=int([4, 64][seed % 2]))
    nrows = F["df_tasks"][(F["df_tasks"][:, 3] & E.DF_LONG) != 0, 3] >> 16
    assert nrows.size and nrows.max() >= 2
