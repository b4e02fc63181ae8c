"""Pins of the oracle's initial perfect matching (greedy maximal matching, then
maximum-cardinality matching by multi-source BFS phases, Sections 5.1-5.2).

Cardinality is pinned to a library Hopcroft-Karp (scipy); maximality of the
greedy step and validity are checked directly; every rule of the reading of
Sections 5.1-5.2 (heavier edges first, equal weights by index, the heavier
BFS parent, the smallest endpoint per tree, a tree stopping at its first
endpoint) is pinned by a hand-derived case whose misreadings change the
matching or the phase and level counts.
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


# ---------------------------------------------------------------------------
# Hand-derived pins of the remaining Phase I rules (the reading of the
# multi-source BFS of Section 5.1 with the "max" parent choice of Section 5.2).
# Each expected matching was worked out by hand, level by level; the comment
# under each case gives what a plausible misreading produces instead.

def test_mcm_endpoint_rule_smallest_row_hand():
    """One tree reaches two unmatched rows at the same level and keeps the
    smaller one.

    Start: col0-row0, col1-row1; columns 2, 3 and rows 2, 3 unmatched.
    Phase 1, level 0: col 2 -> row 0, col 3 -> row 1 (both matched).
    Level 1: frontier cols 0 (tree 2) and 1 (tree 3); rows 2 and 3 are each
    reached from col 0 (w = 4) and col 1 (w = 1): both join tree 2 (heavier
    parent; also the smaller column), which keeps row 2 and augments
    col2-row0-col0-row2.  Tree 3 found nothing.
    Phase 2: col 3 -> row 1 -> col 1 -> {row 2 (matched), row 3 (unmatched)}:
    augment col3-row1-col1-row3.  Result mc = [2, 3, 0, 1], 2 phases, 4 levels.
    Keeping the largest endpoint instead gives mc = [3, 2, 0, 1]."""
    nan = np.nan
    a = np.array([[5.0, nan, 1.0, nan],
                  [nan, 5.0, nan, 1.0],
                  [4.0, 1.0, nan, nan],
                  [4.0, 1.0, nan, nan]])
    wl = from_dense(a)
    mc = np.array([0, 1, -1, -1], dtype=np.int32)
    mr = np.array([0, 1, -1, -1], dtype=np.int32)
    for heavy in (True, False):
        card, mc2, mr2, phases, levels = oracle_mcm(4, wl.col_ptr, wl.row_idx, wl.w, mc, mr, heavy,
                                                    counts=True)
        assert card == 4 and mc2.tolist() == [2, 3, 0, 1], heavy
        assert mr2.tolist() == [2, 3, 0, 1]
        assert (phases, levels) == (2, 4)


def test_mcm_tree_stops_at_first_endpoint_hand():
    """A tree stops growing after the level in which it reaches an unmatched
    row, so it does not compete for rows deeper down.

    Start: col i - row i for i = 0..3; columns 4, 5 and rows 4, 5 unmatched.
    Level 0: col 4 -> row 0 (tree 4), col 5 -> row 2 (tree 5).
    Level 1: col 0 (tree 4) reaches rows 1 and 5; col 2 (tree 5) reaches rows
    3 and 5.  Row 5's parent is col 0 (w = 4 > 1): tree 4 reaches the
    unmatched row 5 and stops, so its matched row 1 is not expanded.
    Level 2: only col 3 (tree 5) expands and reaches the unmatched row 4.
    Both trees augment in one phase: col4-row0-col0-row5 and
    col5-row2-col2-row3-col3-row4, so mc = [5, 1, 3, 4, 0, 2], 1 phase,
    3 levels.  A tree that kept growing would take row 4 through col 1
    (w = 4 > 1), keep it as its smaller endpoint, and leave tree 5 to a
    second phase ending at row 5 through col 2: mc = [1, 4, 5, 3, 0, 2]."""
    nan = np.nan
    a = np.full((6, 6), nan)
    for (r, c, v) in [(0, 0, 5.0), (1, 0, 1.0), (5, 0, 4.0), (1, 1, 5.0), (4, 1, 4.0),
                      (2, 2, 5.0), (3, 2, 1.0), (5, 2, 1.0), (3, 3, 5.0), (4, 3, 1.0),
                      (0, 4, 1.0), (2, 5, 1.0)]:
        a[r, c] = v
    wl = from_dense(a)
    mc = np.array([0, 1, 2, 3, -1, -1], dtype=np.int32)
    mr = np.array([0, 1, 2, 3, -1, -1], dtype=np.int32)
    for heavy in (True, False):
        card, mc2, _, phases, levels = oracle_mcm(6, wl.col_ptr, wl.row_idx, wl.w, mc, mr, heavy,
                                                  counts=True)
        assert card == 6 and mc2.tolist() == [5, 1, 3, 4, 0, 2], heavy
        assert (phases, levels) == (1, 3)
    # both matchings are perfect: the stop rule, not the pattern, decides
    emap = ck.entry_map(wl.col_ptr, wl.row_idx, wl.w)
    assert ck.is_perfect_matching(6, [1, 4, 5, 3, 0, 2], emap)


def test_mcm_singular_phase_counts_hand():
    """A phase that finds no path still counts: rows 0 and 1 are only
    reachable from columns 0 and 1 and column 2 has no entry, so greedy's
    matching is maximum; the one BFS phase from column 2 has an empty first
    frontier expansion (level 0 only) and augments nothing."""
    nan = np.nan
    a = np.array([[1.0, 1.0, nan], [1.0, 1.0, nan], [1.0, 1.0, nan]])
    wl = from_dense(a)
    res = oracle_match(3, wl.col_ptr, wl.row_idx, wl.w)
    assert res.status == -2 and res.mcm_cardinality == 2
    assert (res.greedy_cardinality, res.mcm_phases, res.mcm_levels) == (2, 1, 1)


def test_greedy_equal_weight_ties_hand():
    """Equal weights under the heavy-edge rule: a column proposes to the
    smallest of its heaviest unmatched rows, a row accepts the smallest of its
    heaviest proposers (Section 5.2 prefers heavier edges; ties by index).

    Round 1: col 0 has rows 1 and 2 at w = 3 -> row 1; col 1 has rows 0 and 1
    at w = 3 -> row 0; col 2's heaviest is row 1 (w = 3).  Row 1 gets cols 0
    and 2 at w = 3 and accepts col 0; row 0 accepts col 1.  Round 2: col 2's
    only unmatched row is 2.  Round 3 finds no proposal: mc = [1, 0, 2] after
    3 rounds.  Largest-row ties give [2, 1, 0]; largest-column acceptance
    gives [2, 0, 1]; ignoring the weights gives [0, 1, 2]."""
    a = np.array([[1.0, 3.0, 1.0],
                  [3.0, 3.0, 3.0],
                  [3.0, 1.0, 2.0]])
    wl = from_dense(a)
    card, mc, mr, rounds = oracle_greedy(3, wl.col_ptr, wl.row_idx, wl.w, True, counts=True)
    assert card == 3 and mc.tolist() == [1, 0, 2] and mr.tolist() == [1, 0, 2] and rounds == 3
    card, mc, _, rounds = oracle_greedy(3, wl.col_ptr, wl.row_idx, wl.w, False, counts=True)
    assert card == 3 and mc.tolist() == [0, 1, 2] and rounds == 4
    # all weights equal: both rules reduce to index order
    e = np.full((3, 3), 2.0)
    wl = from_dense(e)
    for heavy in (True, False):
        card, mc, _, rounds = oracle_greedy(3, wl.col_ptr, wl.row_idx, wl.w, heavy, counts=True)
        assert mc.tolist() == [0, 1, 2] and rounds == 4


def test_match_reports_phase1_counts():
    """oracle_match's Phase I counts equal those of its two steps run alone."""
    for seed in range(6):
        wl = small_random(400, 2, 50 + seed)
        gcard, mc, mr, grounds = oracle_greedy(wl.n, wl.col_ptr, wl.row_idx, wl.w, True, counts=True)
        card, _, _, phases, levels = oracle_mcm(wl.n, wl.col_ptr, wl.row_idx, wl.w, mc, mr, True, counts=True)
        res = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w)
        assert (res.greedy_rounds, res.greedy_cardinality, res.mcm_phases, res.mcm_levels) == \
            (grounds, gcard, phases, levels)
        assert res.mcm_cardinality == card
