"""Full-size plan tables of the benchmark workloads, library against oracle, bit for bit,
forward and adjoint (the transposed / reverse-level plans with perm): the 27-point stencil
with off-band entries on 100^3 (SpMV and its lower triangle), the power-law graph of 4M rows
(SpMV), the 27-point Laplacian on 170^3 (SpMV and its lower triangle) and all 256 members of
the batch.  Minutes of CPU time: run with DDF_RUN_SLOW=1."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import ddf
from paper_2111_12243_amd import inputs as I
from test_inspector_parity import assert_same

pytestmark = pytest.mark.slow


def check_full(kind, A):
    p = ddf.ddf_inspect(kind, A, ddf.ddf_opts_default(host_only=1))
    assert_same(ddf.ddf_plan_export(p, 0), O.inspect(kind, A))
    ref, perm = O.inspect_adjoint(kind, A)
    got = ddf.ddf_plan_export(p, 1)
    assert_same(got, ref)
    assert np.array_equal(got["perm"], perm)


@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_workload_tables(name):
    w = I.workload(name)
    check_full(0, w.A)
    if w.L is not None:
        check_full(1, w.L)


def test_batch_member_tables():
    for m in I.workload("c4").batch:
        check_full(1, m["L"])
