"""Executor parity on the GPU through the C ABI: DDF kernels (and the plain comparators)
against the CPU oracle on the same seeded inputs."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rnd(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, shape)


def spmv_case(A, k, seed=0, opts=None, plain=True):
    print(f"spmv n={A.n_rows} m={A.n_cols} nnz={A.nnz} k={k}", flush=True)
    plan = ddf.ddf_inspect(0, A, opts)
    X = rnd((A.n_cols, k), seed)
    G = rnd((A.n_rows, k), seed + 1)
    ref = O.spmv(A, X)
    x, g = dev(X), dev(G)
    y = torch.full((A.n_rows, k), np.nan, dtype=torch.float64, device=DEV)
    ddf.ddf_spmv(plan, x, y, k)
    got = host(y)
    check_product(A, X, got, ref)
    # determinism: a second run is bitwise equal
    y2 = torch.empty_like(y)
    ddf.ddf_spmv(plan, x, y2, k)
    assert np.array_equal(host(y2), got)
    # adjoint
    GX, GV = O.spmv_adj(A, X, G)
    gx = torch.full((A.n_cols, k), np.nan, dtype=torch.float64, device=DEV)
    gv = torch.full((max(A.nnz, 1),), np.nan, dtype=torch.float64, device=DEV)
    vals = dev(A.values) if A.nnz else dev(np.zeros(1))
    ddf.ddf_spmv_adjoint(plan, vals, x, g, gx, gv, k)
    from types import SimpleNamespace
    AT, _ = O.transpose(A)
    check_product(AT, G, host(gx), GX)
    check_gv(A, X, G, host(gv)[:A.nnz], GV)
    if plain:
        yp = torch.empty_like(y)
        ddf.ddf_plain_spmv(plan, vals, x, yp, k)
        check_product(A, X, host(yp), ref)
        gxp = torch.empty_like(gx)
        gvp = torch.empty_like(gv)
        ddf.ddf_plain_spmv_adjoint(plan, vals, x, g, gxp, gvp, k)
        check_product(AT, G, host(gxp), GX)
        check_gv(A, X, G, host(gvp)[:A.nnz], GV)
    return plan


def sptrsv_case(L, k, seed=0, opts=None, plain=True, inplace=False):
    for path in (1, 2, 3):  # multi-block persistent; single-block where eligible; a launch per level
        o = opts if opts is not None else ddf.ddf_opts_default()
        o.solve_path = path
        sptrsv_case_path(L, k, seed, o, plain and path == 1, inplace)


def sptrsv_case_path(L, k, seed, opts, plain, inplace):
    print(f"sptrsv n={L.n_rows} nnz={L.nnz} k={k} path={opts.solve_path}", flush=True)
    plan = ddf.ddf_inspect(1, L, opts)
    B = rnd((L.n_rows, k), seed)
    G = rnd((L.n_rows, k), seed + 1)
    ref = O.sptrsv(L, B)
    b = dev(B)
    x = b if inplace else torch.full_like(b, np.nan)
    ddf.ddf_sptrsv(plan, b, x, k)
    ddf.ddf_plan_sync_status(plan)
    got = host(x)
    check_solve(L, B, got, ref)
    if inplace:
        b = dev(B)
    x2 = torch.empty_like(b)
    ddf.ddf_sptrsv(plan, b, x2, k)
    ddf.ddf_plan_sync_status(plan)
    got2 = host(x2)
    if inplace:
        # an in-place call of the dataflow path runs one launch per level: other rounding order
        check_solve(L, B, got2, ref)
    else:
        assert np.array_equal(got2, got)
    # determinism: the same call again gives the same bits
    x3 = torch.empty_like(b)
    ddf.ddf_sptrsv(plan, b, x3, k)
    assert np.array_equal(host(x3), got2)
    # adjoint
    GB, GV = O.sptrsv_adj(L, ref, G)
    xs, g = dev(ref), dev(G)
    gb = torch.full_like(g, np.nan)
    gv = torch.full((L.nnz,), np.nan, dtype=torch.float64, device=DEV)
    vals = dev(L.values)
    ddf.ddf_sptrsv_adjoint(plan, vals, xs, g, gb, gv, k)
    ddf.ddf_plan_sync_status(plan)
    check_solve(L, G, host(gb), GB, transposed=True)
    check_gv_solve(L, ref, host(gb), GB, host(gv), GV)
    if plain:
        xp = torch.full_like(b, np.nan)
        ddf.ddf_plain_sptrsv(plan, vals, b, xp, k)
        check_solve(L, B, host(xp), ref)
        gbp = torch.full_like(g, np.nan)
        gvp = torch.full_like(gv, np.nan)
        ddf.ddf_plain_sptrsv_adjoint(plan, vals, xs, g, gbp, gvp, k)
        check_solve(L, G, host(gbp), GB, transposed=True)
        check_gv_solve(L, ref, host(gbp), GB, host(gvp), GV)
    return plan


# ---------------------------------------------------------------- crafted

def worked_example():
    rows = np.repeat(np.arange(3), 3)
    return I.csr_from_pairs(3, 8, rows, np.array([0, 2, 5, 1, 3, 6, 2, 4, 7]), np.arange(1.0, 10.0))


def bidiag(n):
    rows = np.concatenate([np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(n - 1), np.arange(n)])
    return I.csr_from_pairs(n, n, rows, cols, np.random.default_rng(n).uniform(1, 2, rows.size))


def test_crafted_spmv():
    spmv_case(worked_example(), 1)
    n = 300
    spmv_case(I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.arange(1.0, n + 1)), 2)
    spmv_case(bidiag(257), 3)
    # a dense row, a giant row, empty rows
    rows = np.concatenate([np.zeros(5000, int), np.arange(2, 60), np.full(3, 70)])
    cols = np.concatenate([np.arange(5000), np.arange(2, 60) * 7, [0, 100, 4999]])
    A = I.csr_from_pairs(80, 5000, rows, cols, np.random.default_rng(0).uniform(-1, 1, rows.size))
    spmv_case(A, 1)
    spmv_case(A, 5)


@pytest.mark.parametrize("window", [128, 1024])
def test_wide_window_stream_tasks(window):
    # diagonal and tridiagonal matrices under windows wider than a wave: rectangular
    # codelets of one or three entries per row run as stream tasks of at most 64 rows
    n = 2000
    opts = ddf.ddf_opts_default(window=window)
    spmv_case(I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.arange(1.0, n + 1)), 1, 11, opts, plain=False)
    tri = I.laplacian(n, 1, 1, [(-1, 0, 0), (0, 0, 0), (1, 0, 0)], 2.0)
    spmv_case(tri, 1, 12, opts, plain=False)


def test_crafted_sptrsv():
    n = 200
    sptrsv_case(I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.arange(1.0, n + 1)), 1)
    sptrsv_case(bidiag(333), 2)
    sptrsv_case(I.tril(I.laplacian(17, 13, 1, I.OFFS_5PT, 4.0)), 1, inplace=True)


def test_c1():
    w = I.c1_laplace2d()
    spmv_case(w.A, 1)
    sptrsv_case(w.L, 1)


@pytest.mark.parametrize("seed", range(12))
def test_random_spmv(seed):
    rng = np.random.default_rng(seed)
    A = I.random_csr(int(rng.integers(1, 400)), int(rng.integers(1, 400)), seed,
                     density=float(rng.uniform(0.002, 0.08)), empty_frac=float(rng.uniform(0, 0.4)),
                     runs=bool(seed % 2))
    k = [1, 2, 3, 8, 13, 32][seed % 6]
    opts = ddf.ddf_opts_default(window=int(rng.choice([8, 64, 100])), ops_per_lane=int(rng.choice([1, 4, 16])),
                                rows_passes=int(rng.choice([1, 2, 4])))
    spmv_case(A, k, seed, opts)


@pytest.mark.parametrize("seed", range(12))
def test_random_sptrsv(seed):
    rng = np.random.default_rng(50 + seed)
    L = I.random_lower(int(rng.integers(1, 300)), seed, density=float(rng.uniform(0.0, 0.05)),
                       runs=bool(seed % 2))
    k = [1, 2, 3, 8, 5, 32][seed % 6]
    opts = ddf.ddf_opts_default(window=int(rng.choice([4, 64])), ops_per_lane=int(rng.choice([1, 4, 16])),
                                rows_passes=int(rng.choice([1, 4])))
    sptrsv_case(L, k, seed, opts, inplace=bool(seed % 3 == 0))


@pytest.mark.parametrize("k", [4, 8])
def test_value_gradient_vector_rhs(k):
    # k = 4 and 8 take the value gradient's 16-byte loads over right-hand sides: rows of ~15
    # entries, then rows past the chunked-row bound (256 entries), then a solve
    for j, dens in enumerate((0.01, 0.25)):
        A = I.random_csr(500, 1500, 70 + j, density=dens, empty_frac=0.1)
        spmv_case(A, k, 70 + j, plain=False)
    sptrsv_case(I.random_lower(700, 80 + k, density=0.05, runs=True), k, 80 + k, plain=False)


@pytest.mark.parametrize("k", [2, 4, 16, 32])
def test_stencil_rhs_counts(k):
    # rectangular shared-offset codelets at every vector right-hand-side count: values staged
    # in LDS where a wave's rows fit (k = 16, 32) and read directly where they do not (k = 2,
    # 4: 64 rows of 27 ops), in the product and in the adjoint's value gradient
    A = I.laplacian(21, 9, 7, I.OFFS_27PT, 26.0)
    spmv_case(A, k, 90 + k, plain=False)


@pytest.mark.parametrize("k", [4, 8])
def test_stencil_factor_uniform_passes(k):
    # stencil factors whose rows are rectangular shared-offset codelets of 3 and 13 ops: with 8
    # right-hand sides each pass holds one task and reads its codelet and column offsets with
    # scalar loads (forward and transposed), with 4 a pass spans two tasks
    offs7 = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    sptrsv_case(I.tril(I.laplacian(11, 9, 13, offs7, 6.0)), k, 110 + k, plain=False)
    sptrsv_case(I.tril(I.laplacian(17, 6, 9, I.OFFS_27PT, 26.0)), k, 120 + k, plain=False)


def off16(a):
    """Device copy of a whose first element sits 8 bytes past a 16-byte boundary."""
    buf = torch.empty(a.size + 1, dtype=torch.float64, device=DEV)
    v = buf[1:]
    v.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()))
    assert v.data_ptr() % 16 == 8
    return v.view(a.shape)


@pytest.mark.parametrize("k", [2, 8])
def test_unaligned_vectors(k):
    # x, y, g and the outputs off 16-byte boundaries: the product takes one right-hand side per
    # lane instead of 16-byte pieces, and the value gradient runs over the CSR pattern instead
    # of the plan; the solve and its adjoint on unaligned vectors too
    A = I.laplacian(13, 7, 5, I.OFFS_27PT, 26.0)
    plan = ddf.ddf_inspect(0, A)
    X, G = rnd((A.n_cols, k), 95), rnd((A.n_rows, k), 96)
    x, g = off16(X), off16(G)
    y = off16(np.full((A.n_rows, k), np.nan))
    ddf.ddf_spmv(plan, x, y, k)
    check_product(A, X, host(y), O.spmv(A, X))
    GX, GV = O.spmv_adj(A, X, G)
    gx = off16(np.full((A.n_cols, k), np.nan))
    gv = off16(np.full(A.nnz, np.nan))
    ddf.ddf_spmv_adjoint(plan, dev(A.values), x, g, gx, gv, k)
    AT, _ = O.transpose(A)
    check_product(AT, G, host(gx), GX)
    check_gv(A, X, G, host(gv), GV)
    L = I.tril(A)
    lp = ddf.ddf_inspect(1, L)
    B = rnd((L.n_rows, k), 97)
    xs = off16(np.full((L.n_rows, k), np.nan))
    ddf.ddf_sptrsv(lp, off16(B), xs, k)
    check_solve(L, B, host(xs), O.sptrsv(L, B))


# ---------------------------------------------------------------- scaled workloads

def test_c2_scaled():
    w = I.c2_stencil27_offband(nx=30)
    spmv_case(w.A, 1)
    sptrsv_case(w.L, 1)
    # small LDS ring: most operands of the single-block solve come through the global gathers
    sptrsv_case(w.L, 1, opts=ddf.ddf_opts_default(thin_ring=256))
    # levels cut into sub-levels of at most 128 lanes
    sptrsv_case(w.L, 1, opts=ddf.ddf_opts_default(thin_lanes=128))


def test_thin_pinned_operands():
    # hub rows read ~30 rows far behind a 256-row ring: operands past two global slots per
    # lane come from pinned LDS entries
    opts = ddf.ddf_opts_default(thin_ring=256)
    sptrsv_case(I.hub_lower(3000, 5), 1, 7, opts)


def test_thin_sub_levels_wide():
    # a 3D 7-point factor whose middle levels are wider than 1024 lanes: single-block only once cut
    offs7 = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    L = I.tril(I.laplacian(48, 48, 48, offs7, 6.0))
    o = ddf.ddf_opts_default(thin_lanes=1024, solve_path=2)
    p = ddf.ddf_inspect(1, L, o)
    assert ddf.ddf_plan_info(p)["solve_path"] == 2
    sptrsv_case_path(L, 1, 0, o, False, False)


def test_c3_scaled():
    w = I.c3_chung_lu(n=200000)
    spmv_case(w.A, 1, plain=True)


def test_c5_scaled():
    w = I.c5_laplace27(nx=32, k=8)
    spmv_case(w.A, 8)
    sptrsv_case(w.L, 8)


@pytest.mark.gpu
@pytest.mark.parametrize("path", [2, 3])
def test_graph_capture_step(path):
    # one step (SpMV, its adjoint, the solve, its adjoint) captured in a graph and replayed
    # several times, with eager work and synchronisation between replays; every replay must
    # match the eager results bit for bit
    print(f"graph capture of one step, solve path {path}", flush=True)
    w = I.c2_stencil27_offband(nx=18)
    A, L = w.A, w.L
    pA = ddf.ddf_inspect(0, A)
    pL = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=path))
    assert ddf.ddf_plan_info(pL)["solve_path"] == path
    vA, vL = dev(A.values), dev(L.values)
    x, gy = dev(rnd((A.n_cols, 1), 3)), dev(rnd((A.n_rows, 1), 4))
    b, gx = dev(rnd((L.n_rows, 1), 5)), dev(rnd((L.n_rows, 1), 6))
    y, gxa, gva = torch.empty_like(gy), torch.empty_like(x), torch.empty(A.nnz, dtype=torch.float64, device=DEV)
    xs, gb, gvl = torch.empty_like(b), torch.empty_like(b), torch.empty(L.nnz, dtype=torch.float64, device=DEV)
    outs = (y, gxa, gva, xs, gb, gvl)

    def step():
        ddf.ddf_spmv_v(pA, vA, x, y, 1)
        ddf.ddf_spmv_adjoint(pA, vA, x, gy, gxa, gva, 1)
        ddf.ddf_sptrsv_v(pL, vL, b, xs, 1)
        ddf.ddf_sptrsv_adjoint(pL, vL, xs, gx, gb, gvl, 1)

    step()
    torch.cuda.synchronize()
    ref = [host(t).copy() for t in outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip(outs, ref):
            assert np.array_equal(host(got), want), f"replay {rep}"
        step()  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.gpu
@pytest.mark.parametrize("path", [1, 2, 3])
def test_forward_and_adjoint_on_two_streams(path):
    # the adjoint's transposed solve runs on a second stream while the forward solve runs;
    # its value gradient waits for the forward solution.  Same bits as the serial calls.
    print(f"two-stream forward and adjoint, solve path {path}", flush=True)
    w = I.c2_stencil27_offband(nx=24)
    L = w.L
    plan = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=path))
    vals, b, g = dev(L.values), dev(rnd((L.n_rows, 1), 7)), dev(rnd((L.n_rows, 1), 8))
    x, gb = torch.empty_like(b), torch.empty_like(b)
    gv = torch.empty(L.nnz, dtype=torch.float64, device=DEV)
    ddf.ddf_sptrsv_v(plan, vals, b, x, 1)
    ddf.ddf_sptrsv_adjoint(plan, vals, x, g, gb, gv, 1)
    ref = (host(x).copy(), host(gb).copy(), host(gv).copy())
    for rep in range(2):
        x2, gb2 = torch.full_like(b, np.nan), torch.full_like(b, np.nan)
        gv2 = torch.full_like(gv, np.nan)
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        with torch.cuda.stream(s1):
            ddf.ddf_sptrsv_v(plan, vals, b, x2, 1)
            done = torch.cuda.Event()
            done.record(s1)
        with torch.cuda.stream(s2):
            ddf.ddf_sptrsv_adjoint(plan, vals, None, g, gb2, None, 1)
            s2.wait_event(done)
            ddf.ddf_sptrsv_value_grad(plan, x2, gb2, gv2, 1)
        torch.cuda.synchronize()
        ddf.ddf_plan_sync_status(plan)
        for got, want in zip((x2, gb2, gv2), ref):
            assert np.array_equal(host(got), want), f"rep {rep}"


@pytest.mark.gpu
def test_value_grad_argument_checks():
    # ddf_sptrsv_value_grad validates before any launch and leaves its output untouched
    print("value-gradient argument checks", flush=True)
    L = I.random_lower(200, 3, density=0.05)
    plan = ddf.ddf_inspect(1, L)
    x, gb = dev(rnd((L.n_rows, 2), 1)), dev(rnd((L.n_rows, 2), 2))
    gv = torch.full((L.nnz,), 7.0, dtype=torch.float64, device=DEV)
    for args, status in (((None, gb, gv, 2), ddf.DDF_E_ARG),   # no x
                         ((x, gb, None, 2), ddf.DDF_E_ARG),    # no output
                         ((x, gb, gb, 2), ddf.DDF_E_ARG),      # output overlaps an input
                         ((x, gb, gv, 0), ddf.DDF_E_ARG)):     # bad right-hand-side count
        with pytest.raises(ddf.DDFError) as e:
            ddf.ddf_sptrsv_value_grad(plan, *args)
        assert e.value.status == status
    assert (host(gv) == 7.0).all()
    spmv_plan = ddf.ddf_inspect(0, L)
    with pytest.raises(ddf.DDFError) as e:
        ddf.ddf_sptrsv_value_grad(spmv_plan, x, gb, gv, 2)
    assert e.value.status == ddf.DDF_E_KIND
    no_adj = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(build_adjoint=0))
    with pytest.raises(ddf.DDFError) as e:
        ddf.ddf_sptrsv_value_grad(no_adj, x, gb, gv, 2)
    assert e.value.status == ddf.DDF_E_UNSUPPORTED
    # a valid call: gv[e] = -<gb[row], x[col]> for every stored entry, the diagonal included
    ddf.ddf_sptrsv_value_grad(plan, x, gb, gv, 2)
    rows = np.repeat(np.arange(L.n_rows), np.diff(L.row_ptr))
    want = -(host(gb)[rows] * host(x)[L.col_idx]).sum(1)
    assert np.allclose(host(gv), want, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- zero diagonals

def same_nonfinite(got, ref, exact_classes):
    """The oracle's non-finite entries (a zero diagonal and every row that depends on it) are
    non-finite on the device too, and the finite ones agree within the solve tolerance.
    exact_classes: also the same inf signs and nans, entry by entry."""
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    if fin.any():
        err = np.max(np.abs(got[fin] - ref[fin]))
        assert err <= 1e-12 * max(np.max(np.abs(ref[fin])), 1e-300)
    if exact_classes:
        assert np.array_equal(got[~fin], ref[~fin], equal_nan=True)


@pytest.mark.parametrize("k", [1, 2])
def test_zero_diagonal_ieee(k):
    # rows with a zero diagonal: forward substitution gives (b - sum) / 0 = +-inf there (the
    # oracle's IEEE rule) and inf or nan in every row that reads them.  The dataflow and
    # per-level kernels divide as the oracle does (same classes); the single-block kernel
    # divides the values first, so the same entries are non-finite, some as nan
    base = I.random_lower(600, 31, density=0.01)
    vals = base.values.copy()
    diag = base.row_ptr[1:] - 1
    vals[diag[[100, 350]]] = 0.0
    L = I.CSR(base.n_rows, base.n_cols, base.row_ptr, base.col_idx, vals)
    rng = np.random.default_rng(4)
    B, G = rng.uniform(-1, 1, (L.n_rows, k)), rng.uniform(-1, 1, (L.n_rows, k))
    with np.errstate(all="ignore"):
        ref = O.sptrsv(L, B)
        lam_ref, _ = O.sptrsv_adj(L, np.nan_to_num(ref), G)
    assert (~np.isfinite(ref)).sum() > 2 and (~np.isfinite(lam_ref)).sum() > 2
    for path in (1, 2, 3):
        print(f"zero diagonal k={k} path={path}", flush=True)
        plan = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=path))
        info = ddf.ddf_plan_info(plan)
        b, x = dev(B), torch.empty((L.n_rows, k), dtype=torch.float64, device=DEV)
        ddf.ddf_sptrsv(plan, b, x, k)
        ddf.ddf_plan_sync_status(plan)
        same_nonfinite(host(x), ref, info["solve_path"] != 2)
        gb = torch.empty_like(x)
        ddf.ddf_sptrsv_adjoint(plan, dev(L.values), None, dev(G), gb, None, k)
        ddf.ddf_plan_sync_status(plan)
        same_nonfinite(host(gb), lam_ref, info["solve_path_adj"] != 2)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_long_rows(k):
    # rows of hundreds of ops run as long-row tasks of the dataflow solve (a wave each), in the
    # forward and the transposed solve
    sptrsv_case(I.long_rows_lower(), k, seed=k)


@pytest.mark.parametrize("k", [1, 4])
def test_wide_rows(k):
    # rows of 17..100 ops: wide-row tasks of several rows each
    sptrsv_case(I.random_lower(300, 44 + k, density=0.2), k, seed=k)


@pytest.mark.parametrize("k", [1, 8])
def test_dataflow_reuses_output_buffer(k):
    # the dataflow solve reads solution values through the caches first: consecutive solves
    # with different right-hand sides into one output buffer must each see only their own
    # values (every launch refills the output with the not-yet-solved mark first)
    L = I.c5_laplace27(nx=24, k=k).L
    o = ddf.ddf_opts_default(solve_path=1, build_adjoint=1)
    plan = ddf.ddf_inspect(1, L, o)
    U, _ = O.transpose(L)
    x = torch.full((L.n_rows, k), np.nan, dtype=torch.float64, device=DEV)
    lam = torch.full_like(x, np.nan)
    vals = dev(L.values)
    for rep in range(4):
        B = rnd((L.n_rows, k), 100 + rep) * (rep + 1)
        ddf.ddf_sptrsv(plan, dev(B), x, k)
        ref = O.sptrsv(L, B)
        check_solve(L, B, host(x), ref)
        G = rnd((L.n_rows, k), 200 + rep)
        ddf.ddf_sptrsv_adjoint(plan, vals, x, dev(G), lam, None, k)
        check_solve(L, G, host(lam), O.sptrsv_adj(L, ref, G)[0], transposed=True)
    ddf.ddf_plan_sync_status(plan)


@pytest.mark.parametrize("k", [1, 8])
def test_spin_limit_watchdog(k):
    # a spin limit of one poll: the dataflow solve's first wait trips the watchdog, every wave
    # stops waiting and the kernel ends; the call is then reported invalid, the flag cleared,
    # and the next solve at the default limit is exact again (the wait is bounded by the
    # limit, so this never hangs)
    L = bidiag(20000)
    plan = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=1))
    B = rnd((L.n_rows, k), k)
    b = dev(B)
    x = torch.full_like(b, np.nan)
    ddf.ddf_plan_set_spin_limit(plan, 1)
    ddf.ddf_sptrsv(plan, b, x, k)
    with pytest.raises(ddf.DDFError) as err:
        ddf.ddf_plan_sync_status(plan)
    assert err.value.status == ddf.DDF_E_DEVICE
    ddf.ddf_plan_set_spin_limit(plan, 0)
    x = torch.full_like(b, np.nan)
    ddf.ddf_sptrsv(plan, b, x, k)
    ddf.ddf_plan_sync_status(plan)
    check_solve(L, B, host(x), O.sptrsv(L, B))
