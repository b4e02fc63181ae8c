"""Independent checkers used to pin the oracle and the GPU results.

These work from the matching as a permutation of columns (perm[j] = row
matched to column j) and enumerate pairs of columns directly, a different
formulation from the oracle's row scan, so a mistake in one is unlikely to
be repeated in the other.  Exact sums use fractions.Fraction (every binary64
value is a rational number).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def entry_map(col_ptr, row_idx, w):
    """{(row, col): (weight, position)} for a small CSC."""
    m = {}
    n = len(col_ptr) - 1
    for c in range(n):
        for k in range(int(col_ptr[c]), int(col_ptr[c + 1])):
            m[(int(row_idx[k]), c)] = (float(w[k]), k)
    return m


def is_perfect_matching(n, perm, emap) -> bool:
    perm = [int(x) for x in perm]
    if len(perm) != n or sorted(perm) != list(range(n)):
        return False
    return all((perm[j], j) in emap for j in range(n))


def exact_weight(perm, emap) -> Fraction:
    return sum((Fraction(emap[(int(r), j)][0]) for j, r in enumerate(perm)), Fraction(0))


def pair_gain(perm, emap, j, c):
    """Gain of swapping the rows of columns j and c (an alternating 4-cycle),
    evaluated as (w(i,j) + w(m_j,m_i)) - (w(i,m_i) + w(m_j,j)) with i = perm[c],
    m_j = perm[j], m_i = c.  None if one of the two new edges is absent."""
    mj, i = int(perm[j]), int(perm[c])
    if (i, j) not in emap or (mj, c) not in emap:
        return None
    return (emap[(i, j)][0] + emap[(mj, c)][0]) - (emap[(i, c)][0] + emap[(mj, j)][0])


def positive_4cycles(n, perm, emap):
    """All column pairs (j, c), j < c, whose swap has a positive gain."""
    out = []
    for j in range(n):
        for c in range(j + 1, n):
            g = pair_gain(perm, emap, j, c)
            if g is not None and g > 0.0:
                out.append((j, c, g))
    return out


def brute_force_optimum(n, emap):
    """Maximum exact weight over all perfect matchings (n <= 8), or None."""
    best = None
    for p in itertools.permutations(range(n)):
        # p[j] = row of column j
        if all((p[j], j) in emap for j in range(n)):
            wsum = sum((Fraction(emap[(p[j], j)][0]) for j in range(n)), Fraction(0))
            if best is None or wsum > best:
                best = wsum
    return best


def one_round_by_pairs(n, perm, emap):
    """One bulk-synchronous WIAC round derived from column pairs.

    A 4-cycle is an unordered pair of columns {a, b} whose rows can be
    exchanged.  Its root is the column whose matched row is smaller (rows
    i > m_j only), the other column is the one whose matched row is larger.
    Step C keeps, per root, the positive cycle of largest gain (ties: smaller
    row of the other column, i.e. the row i of the cycle).  Step D keeps, per
    other column, the largest-gain root (ties: smaller root) unless that other
    column is itself a root with a kept cycle.  Returns (new_perm,
    n_candidates, n_applied)."""
    perm = [int(x) for x in perm]
    kept = {}  # root -> (g, i, other)
    for a in range(n):
        for b in range(n):
            if a == b or perm[b] <= perm[a]:
                continue
            root, other = a, b  # perm[root] < perm[other]
            g = pair_gain(perm, emap, root, other)
            if g is None or not g > 0.0:
                continue
            i = perm[other]
            cur = kept.get(root)
            if cur is None or g > cur[0] or (g == cur[0] and i < cur[1]):
                kept[root] = (g, i, other)
    accepted = {}
    for root, (g, i, other) in kept.items():
        if other in kept:
            continue
        cur = accepted.get(other)
        if cur is None or g > cur[0] or (g == cur[0] and root < cur[1]):
            accepted[other] = (g, root)
    new = list(perm)
    for other, (g, root) in accepted.items():
        new[root], new[other] = perm[other], perm[root]
    return new, len(kept), len(accepted)


def round_is_disjoint_positive_swaps(n, before, after, emap) -> bool:
    """The columns whose row changed pair up into row exchanges, each of
    positive gain with respect to `before` (vertex-disjoint 4-cycles)."""
    before = [int(x) for x in before]
    after = [int(x) for x in after]
    changed = [j for j in range(n) if before[j] != after[j]]
    col_of_row_before = {r: j for j, r in enumerate(before)}
    seen = set()
    for j in changed:
        if j in seen:
            continue
        c = col_of_row_before[after[j]]
        if c == j or after[c] != before[j]:
            return False
        g = pair_gain(before, emap, j, c)
        if g is None or not g > 0.0:
            return False
        seen.update((j, c))
    return len(seen) == len(changed)


def dense_from_workload(wl):
    a = np.full((wl.n, wl.n), np.nan)
    for c in range(wl.n):
        for k in range(int(wl.col_ptr[c]), int(wl.col_ptr[c + 1])):
            a[wl.row_idx[k], c] = wl.w[k]
    return a
