"""CPU tests of the seeded input generators: the sizes and structure each
recipe states, a well-formed CSC, the planted perfect matching inside the
pattern, the value ranges, and determinism under fixed seeds."""
import math

import numpy as np
import pytest

from workloads import poisson_arrivals, random_matrix, rmat, serving_matrix, small_random, stencil27, workload

LN10 = math.log(10.0)


def _check_csc(wl):
    """Well-formed CSC (rows in range, strictly increasing per column), finite
    weights, and the planted matching is a permutation of entries; returns
    the column of every entry and the positions of the planted entries."""
    n = wl.n
    assert wl.col_ptr.dtype == np.int64 and wl.row_idx.dtype == np.int32 and wl.w.dtype == np.float64
    assert wl.col_ptr.size == n + 1 and wl.col_ptr[0] == 0 and wl.col_ptr[-1] == wl.nnz
    assert np.all(np.diff(wl.col_ptr) >= 0)
    assert wl.nnz == 0 or (wl.row_idx.min() >= 0 and wl.row_idx.max() < n)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(wl.col_ptr))
    key = cols * n + wl.row_idx
    assert np.all(np.diff(key) > 0)
    assert np.all(np.isfinite(wl.w))
    assert np.array_equal(np.sort(wl.planted), np.arange(n))
    want = np.arange(n, dtype=np.int64) * n + wl.planted
    pos = np.minimum(np.searchsorted(key, want), max(wl.nnz - 1, 0))
    assert np.array_equal(key[pos], want), "planted matching leaves the pattern"
    return cols, pos


def test_small_case_recipe():
    wl = workload(0)
    assert (wl.n, wl.nnz) == (2000, 17965)
    _check_csc(wl)
    deg = np.diff(wl.col_ptr)
    assert deg.min() >= 1 and deg.max() <= 9  # 8 draws with replacement + the diagonal
    assert wl.w.min() >= -3 * LN10 and wl.w.max() <= 3 * LN10  # ln of 10^U(-3, 3)


def test_random_generator_deterministic():
    a = random_matrix(500, 6, 11, 12, 13)
    b = random_matrix(500, 6, 11, 12, 13)
    c = random_matrix(500, 6, 11, 12, 14)
    for x, y in ((a.col_ptr, b.col_ptr), (a.row_idx, b.row_idx), (a.w, b.w), (a.planted, b.planted)):
        assert np.array_equal(x, y)
    assert not np.array_equal(a.planted, c.planted)  # another row permutation
    # the permutation moves rows only: column counts are the same
    assert np.array_equal(a.col_ptr, c.col_ptr)


@pytest.mark.parametrize("g", [3, 6])
def test_stencil_recipe(g):
    wl = stencil27(g, g, g, 5, 6)
    n = g ** 3
    assert wl.n == n and wl.nnz == (3 * g - 2) ** 3  # pairs of grid points within one step per axis
    _, pos = _check_csc(wl)
    deg = np.diff(wl.col_ptr)
    assert deg.max() == 27 and deg.min() == 8  # interior and corner vertices
    assert deg[0] == 8 and deg[1 + g * (1 + g)] == 27
    diag = np.zeros(wl.nnz, dtype=bool)
    diag[pos] = True  # the planted entries are the permuted diagonal
    assert wl.w[diag].min() >= math.log(1e-6) and wl.w[diag].max() <= math.log(10.0)
    assert wl.w[~diag].min() >= -4 * LN10 and wl.w[~diag].max() <= 0.0


def test_stencil_leading_block():
    wl = stencil27(5, 5, 5, 1, 2, n_keep=37)
    assert wl.n == 37
    _check_csc(wl)


def test_rmat_recipe():
    scale, ef = 10, 8
    wl = rmat(scale, ef, 21, 22, 23)
    n = 1 << scale
    assert wl.n == n and n < wl.nnz <= n * ef + n  # duplicates removed, identity added
    _check_csc(wl)
    deg = np.diff(wl.col_ptr)
    # destination bit 0 has probability a + c = 0.76 at every level, so
    # column 0 is the hub and the degrees are far from uniform
    assert int(np.argmax(deg)) == 0 and deg[0] > 10 * deg.mean()
    assert np.array_equal(rmat(scale, ef, 21, 22, 23).row_idx, wl.row_idx)


def test_small_random_integer_weights():
    wl = small_random(300, 4, 9, integer_weights=True, weight_range=2)
    _check_csc(wl)
    assert set(np.unique(wl.w)).issubset({-2.0, -1.0, 0.0, 1.0, 2.0})


def test_serving_stream_recipe():
    for i in range(12):
        wl = serving_matrix(i)
        assert 100 <= wl.n <= 100000
        _check_csc(wl)
        again = serving_matrix(i)
        assert np.array_equal(again.row_idx, wl.row_idx) and np.array_equal(again.w, wl.w)


def test_poisson_arrivals():
    t = poisson_arrivals(20000, 50.0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1.0 / 50.0) < 0.05 / 50.0  # mean gap 1/rate, within 5%
    assert np.array_equal(t, poisson_arrivals(20000, 50.0))
