"""Oracle levels (ASAP dependence levels of forward substitution) against closed forms and a
brute-force longest path."""
import functools

import numpy as np
import pytest

import oracle as O
from paper_2111_12243_amd import inputs as I


def grid_lower(nx, ny, nz, offs):
    rp, col, _ = I.stencil_pattern(nx, ny, nz, I.lower_offsets(offs))
    return I.CSR(nx * ny * nz, nx * ny * nz, rp.astype(np.int32), col, np.ones(col.size))


OFFS_7PT = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_identity_and_bidiagonal():
    n = 17
    eye = I.csr_from_pairs(n, n, np.arange(n), np.arange(n), np.ones(n))
    lev, nl = O.levels(eye)
    assert nl == 1 and np.all(lev == 0)
    rows = np.concatenate([np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(n - 1), np.arange(n)])
    bi = I.csr_from_pairs(n, n, rows, cols, np.ones(rows.size))
    lev, nl = O.levels(bi)
    assert nl == n and np.array_equal(lev, np.arange(n))


@pytest.mark.parametrize("N", [5, 16, 64])
def test_2d_5pt_levels(N):
    lev, nl = O.levels(grid_lower(N, N, 1, I.OFFS_5PT))
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    assert np.array_equal(lev, (i + j).ravel())
    assert nl == 2 * N - 1


def test_c1_levels():
    lev, nl = O.levels(I.c1_laplace2d().L)
    assert nl == 127


@pytest.mark.parametrize("shape", [(4, 5, 6), (7, 3, 2)])
def test_3d_7pt_levels(shape):
    nx, ny, nz = shape
    offs = sorted(OFFS_7PT, key=lambda o: (o[2], o[1], o[0]))
    lev, nl = O.levels(grid_lower(nx, ny, nz, offs))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    assert np.array_equal(lev, (i + j + k).ravel())


@pytest.mark.parametrize("shape", [(5, 5, 5), (6, 4, 3), (10, 10, 10)])
def test_3d_27pt_levels(shape):
    nx, ny, nz = shape
    lev, nl = O.levels(grid_lower(nx, ny, nz, I.OFFS_27PT))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    assert np.array_equal(lev, (i + 2 * j + 4 * k).ravel())
    assert nl == (nx - 1) + 2 * (ny - 1) + 4 * (nz - 1) + 1


def test_27pt_level_count_formula_large():
    # 170^3 grid: (169) + 2*169 + 4*169 + 1 = 1184 levels; checked on the formula's
    # building block, a thin slab whose count the same formula gives
    lev, nl = O.levels(grid_lower(170, 3, 2, I.OFFS_27PT))
    assert nl == 169 + 2 * 2 + 4 * 1 + 1


@pytest.mark.parametrize("seed", range(8))
def test_bruteforce_longest_path(seed):
    L = I.random_lower(40, seed, density=0.15)
    preds = [[int(c) for c in L.col_idx[L.row_ptr[i]:L.row_ptr[i + 1]] if c != i]
             for i in range(L.n_rows)]

    @functools.lru_cache(None)
    def longest_chain_ending_at(i):  # number of edges on the longest path ending at i
        return max((1 + longest_chain_ending_at(p) for p in preds[i]), default=0)

    lev, nl = O.levels(L)
    assert [longest_chain_ending_at(i) for i in range(L.n_rows)] == lev.tolist()
    # invariants: dependences point strictly down; ASAP is tight
    for i in range(L.n_rows):
        for p in preds[i]:
            assert lev[p] < lev[i]
        if lev[i] > 0:
            assert max(lev[p] for p in preds[i]) == lev[i] - 1
