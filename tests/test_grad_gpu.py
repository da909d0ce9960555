"""Autograd wrappers: gradcheck in float64 on small systems, and gradients against the
oracle's adjoints and closed forms."""
import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_12243_amd import autograd, ddf  # noqa: E402

DEV = "cuda:0"


def test_spmv_gradcheck():
    A = I.random_csr(30, 25, 3, density=0.2, empty_frac=0.1)
    plan = ddf.ddf_inspect(0, A)
    v = torch.tensor(A.values, device=DEV, requires_grad=True)
    x = torch.tensor(np.random.default_rng(0).uniform(-1, 1, (25, 3)), device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda v_, x_: autograd.spmv(plan, v_, x_), (v, x), eps=1e-6, atol=1e-9)


def test_sptrsv_gradcheck():
    L = I.random_lower(35, 4, density=0.15)
    plan = ddf.ddf_inspect(1, L)
    v = torch.tensor(L.values, device=DEV, requires_grad=True)
    b = torch.tensor(np.random.default_rng(1).uniform(-1, 1, (35, 2)), device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda v_, b_: autograd.sptrsv(plan, v_, b_), (v, b), eps=1e-6, atol=1e-8)


def test_vector_rhs_and_closed_form():
    n = 40
    d = np.random.default_rng(2).uniform(0.5, 2, n)
    D = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), d)
    plan = ddf.ddf_inspect(1, D)
    v = torch.tensor(d, device=DEV, requires_grad=True)
    b = torch.tensor(np.random.default_rng(3).uniform(-1, 1, n), device=DEV, requires_grad=True)
    g = torch.tensor(np.random.default_rng(4).uniform(-1, 1, n), device=DEV)
    x = autograd.sptrsv(plan, v, b)
    (x * g).sum().backward()
    assert np.allclose(b.grad.cpu().numpy(), g.cpu().numpy() / d, rtol=1e-15, atol=0)
    assert np.allclose(v.grad.cpu().numpy(), -g.cpu().numpy() * b.detach().cpu().numpy() / d ** 2, rtol=1e-14)


def test_c1_grads_match_oracle():
    w = I.c1_laplace2d()
    plan = ddf.ddf_inspect(0, w.A)
    v = torch.tensor(w.A.values, device=DEV, requires_grad=True)
    x = torch.tensor(w.X, device=DEV, requires_grad=True)
    y = autograd.spmv(plan, v, x)
    (y * torch.tensor(w.Gy, device=DEV)).sum().backward()
    GX, GV = O.spmv_adj(w.A, w.X, w.Gy)
    assert np.max(np.abs(x.grad.cpu().numpy() - GX)) <= 1e-13
    assert np.max(np.abs(v.grad.cpu().numpy() - GV)) <= 1e-13
