"""The C ABI without a GPU: the library loads, exports what include/ddf.h declares, and
rejects bad input before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2111_12243_amd import ddf
from paper_2111_12243_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "ddf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ddf_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = declared()
    assert len(names) >= 25
    lib = ctypes.CDLL(ddf.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(ddf.EXPORTED) == names


def test_status_strings_and_version():
    assert ddf.ddf_status_string(0) == "DDF_OK"
    assert ddf.ddf_status_string(8) == "DDF_E_DEVICE"
    assert ddf.ddf_version().startswith("ddf")


def test_defaults():
    o = ddf.ddf_opts_default()
    assert (o.window, o.build_adjoint, o.host_only) == (64, 1, 0)


def expect(status, fn):
    with pytest.raises(ddf.DDFError) as e:
        fn()
    assert e.value.status == status, str(e.value)


def hopts():
    return ddf.ddf_opts_default(host_only=1)


def test_malformed_csr_rejected():
    good = I.random_csr(20, 20, 1, density=0.3)
    bad = I.CSR(20, 20, good.row_ptr.copy(), good.col_idx.copy(), good.values)
    bad.row_ptr[5] = bad.row_ptr[6] + 1
    expect(ddf.DDF_E_CSR, lambda: ddf.ddf_inspect(0, bad, hopts()))
    bad = I.CSR(20, 20, good.row_ptr, good.col_idx.copy(), good.values)
    bad.col_idx[0] = 25
    expect(ddf.DDF_E_CSR, lambda: ddf.ddf_inspect(0, bad, hopts()))
    bad = I.CSR(20, 20, good.row_ptr, good.col_idx.copy(), good.values)
    r = int(np.argmax(np.diff(good.row_ptr) >= 2))
    s = good.row_ptr[r]
    bad.col_idx[s], bad.col_idx[s + 1] = good.col_idx[s + 1], good.col_idx[s]
    expect(ddf.DDF_E_CSR, lambda: ddf.ddf_inspect(0, bad, hopts()))
    bad.col_idx[s + 1] = bad.col_idx[s]  # repeated column
    expect(ddf.DDF_E_CSR, lambda: ddf.ddf_inspect(0, bad, hopts()))


def test_triangular_checks():
    A = I.random_csr(10, 10, 3, density=0.5, empty_frac=0.0)
    expect(ddf.DDF_E_NOT_LOWER, lambda: ddf.ddf_inspect(1, A, hopts()))
    L = I.random_lower(10, 2)
    rows = np.repeat(np.arange(10), np.diff(L.row_ptr))
    keep = ~((rows == 4) & (L.col_idx == 4))
    nod = I.csr_from_pairs(10, 10, rows[keep], L.col_idx[keep], L.values[keep])
    expect(ddf.DDF_E_NO_DIAG, lambda: ddf.ddf_inspect(1, nod, hopts()))
    rect = I.CSR(10, 11, L.row_ptr, L.col_idx, L.values)
    expect(ddf.DDF_E_ARG, lambda: ddf.ddf_inspect(1, rect, hopts()))
    expect(ddf.DDF_E_KIND, lambda: ddf.ddf_inspect(7, L, hopts()))


def test_options_checked():
    L = I.random_lower(10, 2)
    expect(ddf.DDF_E_ARG, lambda: ddf.ddf_inspect(1, L, ddf.ddf_opts_default(host_only=1, window=4096)))
    expect(ddf.DDF_E_ARG, lambda: ddf.ddf_inspect_batch(1, [L, L], [1, 33], hopts()))
    expect(ddf.DDF_E_KIND, lambda: ddf.ddf_inspect_batch(0, [L], [1], hopts()))


def test_host_only_plan_refuses_execution():
    p = ddf.ddf_inspect(1, I.random_lower(10, 2), hopts())
    expect(ddf.DDF_E_UNSUPPORTED, lambda: ddf.ddf_sptrsv_v(p, 0, 0, 0, 1, 0))
    expect(ddf.DDF_E_UNSUPPORTED, lambda: ddf.ddf_spmv_v(p, 0, 0, 0, 1, 0))
    expect(ddf.DDF_E_UNSUPPORTED, lambda: ddf.ddf_sptrsv_value_grad(p, 0, 0, 0, 1, 0))
    q = ddf.ddf_inspect(0, I.random_csr(8, 8, 1), ddf.ddf_opts_default(host_only=1, build_adjoint=0))
    expect(ddf.DDF_E_UNSUPPORTED, lambda: ddf.ddf_plan_export(q, 1))
    info = ddf.ddf_plan_info(p)
    assert info["n_tasks"] > 0 and info["has_adjoint"] == 1  # tables are built, not uploaded


def test_batch_host_plan_members_match_single():
    mats = [I.batch_matrix(b, n_lo=300, n_hi=3000)["L"] for b in range(4)]
    p = ddf.ddf_inspect_batch(1, mats, [1, 2, 3, 4], hopts())
    for b, L in enumerate(mats):
        single = ddf.ddf_plan_export(ddf.ddf_inspect(1, L, hopts()), 0)
        mine = ddf.ddf_plan_export(p, 0, b)
        for k in single:
            assert np.array_equal(single[k], mine[k])


def test_traffic_formulas():
    w = I.c1_laplace2d()
    p = ddf.ddf_inspect(0, w.A, hopts())
    ba, bc, fl = ddf.ddf_plan_traffic(p, ddf.DDF_OP_SPMV, 1)
    n, nnz = w.A.n_rows, w.A.nnz
    assert bc == 12 * nnz + 4 * (n + 1) + 16 * n
    assert fl == 2 * nnz
    info = ddf.ddf_plan_info(p)
    assert info["dev_plan_bytes"] > 0
    # values + vectors + the tables one launch reads: records and aux of the codelets it runs as
    # codelets, its tasks, and columns and row pointers of the rows it runs from the CSR pattern
    D = ddf.ddf_plan_device_tables(p, 0)
    cods, aux, tasks = D["cods"], D["aux"], D["tasks"]
    offs = cods[:, 10:15]
    starts = [min([o for o in r if o >= 0], default=None) for r in offs]
    ends, nxt = [0] * len(starts), aux.size
    for c in range(len(starts) - 1, -1, -1):
        ends[c] = nxt
        if starts[c] is not None:
            nxt = starts[c]
    tables, csr_rows, csr_nnz = tasks.shape[0] * 16, 0, 0
    from_csr = (1 << 11) | (1 << 13)
    run_as_codelet = set(int(t[0]) for t in tasks if not t[3] & from_csr)
    for c in run_as_codelet:
        tables += 64 + 4 * (ends[c] - starts[c] if starts[c] is not None else 0)
    rows = [r for t in tasks if t[3] & (1 << 11) for r in range(t[1], t[2])]
    rows += [int(r) for t in tasks if t[3] & (1 << 13) for r in D["rowlist"][t[1]:t[2]]]
    tables += 4 * D["rowlist"].size
    csr_rows = len(rows)
    csr_nnz = sum(int(w.A.row_ptr[r + 1] - w.A.row_ptr[r]) for r in rows)
    assert ba == 8 * nnz + 16 * n + tables + 4 * csr_nnz + 8 * csr_rows


def test_row_list_tasks():
    # scattered short rows of small codelets run from the CSR pattern, 64 rows to a wave
    from paper_2111_12243_amd import inputs as I2
    A = I2.c3_chung_lu(n=20000).A
    p = ddf.ddf_inspect(0, A, hopts())
    D = ddf.ddf_plan_device_tables(p, 0)
    rl = D["rowlist"]
    tasks = D["tasks"]
    rt = tasks[(tasks[:, 3] & (1 << 13)) != 0]
    assert rl.size > 0 and rt.shape[0] == (rl.size + 63) // 64
    lens = np.diff(A.row_ptr)[rl]
    assert (lens <= 8).all() and (np.diff(lens) >= 0).all()  # sorted by length
    assert np.array_equal(np.sort(np.concatenate([np.arange(t[1], t[2]) for t in rt])), np.arange(rl.size))
