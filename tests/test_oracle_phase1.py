"""Pins of the oracle's initial perfect matching (greedy maximal matching, then
maximum-cardinality matching by multi-source BFS phases, Sections 5.1-5.2).

Cardinality is pinned to a library Hopcroft-Karp (scipy); maximality of the
greedy step and validity are checked directly; the heavy-edge tie-break is
pinned on hand-derived cases.  Which maximum matching the BFS phases return
beyond that is a reading of Section 5.2 (parity unpinned).
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import maximum_bipartite_matching

from oracle import oracle_greedy, oracle_match, oracle_mcm
from tests import checkers as ck
from workloads import from_dense, small_random


def _library_cardinality(wl):
    a = sp.csc_matrix((np.ones(wl.nnz), wl.row_idx, wl.col_ptr), shape=(wl.n, wl.n))
    m = maximum_bipartite_matching(a.tocsr(), perm_type="column")
    return int((m >= 0).sum())


def _drop_diag(wl, frac, seed):
    """Remove a fraction of the planted entries so the matrix may be singular."""
    rng = np.random.default_rng(seed)
    keep = np.ones(wl.nnz, dtype=bool)
    for j in range(wl.n):
        if rng.random() < frac:
            lo, hi = wl.col_ptr[j], wl.col_ptr[j + 1]
            k = lo + np.searchsorted(wl.row_idx[lo:hi], wl.planted[j])
            keep[k] = False
    counts = np.array([keep[wl.col_ptr[j]:wl.col_ptr[j + 1]].sum() for j in range(wl.n)])
    col_ptr = np.zeros(wl.n + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum(counts)
    return type(wl)(wl.name + "_holes", wl.n, col_ptr, wl.row_idx[keep], wl.w[keep], wl.planted)


@pytest.mark.parametrize("n,d,seed,holes", [(30, 1, 1, 0.0), (200, 2, 2, 0.0), (500, 1, 3, 0.3),
                                            (500, 3, 4, 0.5), (1000, 2, 5, 0.2), (64, 1, 6, 0.9)])
@pytest.mark.parametrize("heavy", [True, False])
def test_greedy_maximal_and_mcm_maximum(n, d, seed, holes, heavy):
    wl = small_random(n, d, seed)
    if holes:
        wl = _drop_diag(wl, holes, seed)
    emap = ck.entry_map(wl.col_ptr, wl.row_idx, wl.w)
    card, mc, mr = oracle_greedy(wl.n, wl.col_ptr, wl.row_idx, wl.w, heavy)
    # a valid matching inside the pattern
    assert card == int((mc >= 0).sum()) == int((mr >= 0).sum())
    for j in range(n):
        if mc[j] >= 0:
            assert (int(mc[j]), j) in emap and mr[mc[j]] == j
    # maximal: no edge joins an unmatched row and an unmatched column
    assert not any(mc[c] < 0 and mr[r] < 0 for (r, c) in emap)
    card2, mc2, mr2 = oracle_mcm(wl.n, wl.col_ptr, wl.row_idx, wl.w, mc, mr, heavy)
    assert card2 == _library_cardinality(wl)
    for j in range(n):
        if mc2[j] >= 0:
            assert (int(mc2[j]), j) in emap and mr2[mc2[j]] == j
    res = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w, heavy)
    if card2 == n:
        assert res.status == 0 and ck.is_perfect_matching(n, res.perm, emap)
        assert ck.positive_4cycles(n, res.perm, emap) == [] if n <= 200 else True
    else:
        assert res.status == -2 and (res.perm == -1).all()


def test_greedy_heavy_tiebreak_hand():
    # Section 5.2: the greedy step prefers heavier edges.  Column 0 proposes to
    # its heaviest row 1 (w=5), column 1 to its heaviest row 1 (w=7); row 1
    # accepts the heavier proposer, column 1.  Next round column 0 proposes to
    # row 0, its only unmatched neighbour.
    a = np.array([[1.0, 2.0], [5.0, 7.0]])
    wl = from_dense(a)
    card, mc, mr = oracle_greedy(2, wl.col_ptr, wl.row_idx, wl.w, True)
    assert card == 2 and mc.tolist() == [0, 1]
    # without the heuristic, index order decides: column 0 and column 1 both
    # propose to row 0, which accepts column 0; then column 1 takes row 1
    card, mc, mr = oracle_greedy(2, wl.col_ptr, wl.row_idx, wl.w, False)
    assert card == 2 and mc.tolist() == [0, 1]
    b = np.array([[1.0, 9.0], [5.0, 2.0]])
    wl = from_dense(b)
    card, mc, _ = oracle_greedy(2, wl.col_ptr, wl.row_idx, wl.w, True)
    assert mc.tolist() == [1, 0]  # col 0 -> row 1 (5), col 1 -> row 0 (9)


def test_mcm_heavy_parent_hand():
    # Two augmenting paths from the unmatched column 2 (Section 5.2, the "max"
    # semiring picks the heavier edge when a row can be reached two ways).
    # Matching after greedy: col0-row0, col1-row1; col 2 and row 2 unmatched.
    # Column 2 reaches rows 0 and 1; row 0 leads to col 0 which reaches row 2,
    # row 1 leads to col 1 which also reaches row 2.  Row 2 is reached at the
    # second level from cols 0 and 1; the heavier edge (col 1, w=8) is its parent.
    nan = np.nan
    a = np.array([[5.0, nan, 1.0],
                  [nan, 5.0, 1.0],
                  [3.0, 8.0, nan]])
    wl = from_dense(a)
    mc = np.array([0, 1, -1], dtype=np.int32)
    mr = np.array([0, 1, -1], dtype=np.int32)
    card, mc2, mr2 = oracle_mcm(3, wl.col_ptr, wl.row_idx, wl.w, mc, mr, True)
    assert card == 3 and mc2.tolist() == [0, 2, 1]
    card, mc3, _ = oracle_mcm(3, wl.col_ptr, wl.row_idx, wl.w, mc, mr, False)
    assert card == 3 and mc3.tolist() == [2, 1, 0]  # index order: parent col 0


def test_singular_structurally():
    nan = np.nan
    a = np.array([[1.0, 1.0, nan], [1.0, 1.0, nan], [1.0, 1.0, nan]])
    wl = from_dense(a)
    res = oracle_match(3, wl.col_ptr, wl.row_idx, wl.w)
    assert res.status == -2 and res.mcm_cardinality == 2
