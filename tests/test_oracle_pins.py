"""Pins of the CPU oracle against what the paper and the mathematics fix.

* hand-derived cases (tests/golden/wiac_cases.json, tree_sum_cases.json);
* brute force over all perfect matchings for n <= 8;
* one round re-derived from column pairs (tests/checkers.py);
* invariants at any size: validity, strict exact-weight increase per round,
  vertex-disjoint positive swaps per round, no positive 4-cycle at the end;
* the pairwise-summation error bound for the total weight;
* a library assignment solver as the optimum for moderate n.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle_improve, oracle_tree_sum
from tests import checkers as ck
from workloads import from_dense, small_random

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _dense(rows):
    return np.array([[np.nan if v is None else float(v) for v in r] for r in rows])


def _f(v):
    return float(v)  # strings carry signed zeros ("-0.0") through JSON


# --------------------------------------------------------------------------
# total-weight summation order

@pytest.mark.parametrize("case", _load("tree_sum_cases.json")["cases"])
def test_tree_sum_golden(case):
    x = np.array([_f(v) for v in case["x"]], dtype=np.float64)
    got = oracle_tree_sum(x)
    exp = _f(case["expected"])
    assert got == exp and math.copysign(1.0, got) == math.copysign(1.0, exp), case["why"]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 1000, 4097])
def test_tree_sum_error_bound(n):
    # pairwise summation: |s - exact| <= ceil(log2 n) * u * sum|x| (Higham, ch. 4)
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
    got = Fraction(oracle_tree_sum(x))
    exact = sum((Fraction(v) for v in x), Fraction(0))
    levels = max(1, math.ceil(math.log2(n)))
    bound = Fraction(levels) * Fraction(2.0 ** -53) * sum((abs(Fraction(v)) for v in x), Fraction(0))
    assert abs(got - exact) <= bound * Fraction(1001, 1000)


def test_tree_sum_integers_exact():
    x = np.arange(-5000, 7001, dtype=np.float64)
    assert oracle_tree_sum(x) == float(x.astype(np.int64).sum())


# --------------------------------------------------------------------------
# hand-derived WIAC cases

@pytest.mark.parametrize("case", _load("wiac_cases.json")["cases"], ids=lambda c: c["name"])
def test_wiac_golden(case):
    wl = from_dense(_dense(case["dense"]), planted=case["mate_in"])
    # an unbounded run is capped at 1000 rounds so a non-terminating loop fails
    r = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, case["max_rounds"] or 1000)
    assert r.status == 0
    assert r.perm.tolist() == case["expected_perm"], case["why"]
    assert r.total == case["expected_total"]
    assert r.rounds == case["expected_rounds"]
    assert r.round_candidates == case["expected_candidates"]
    assert r.round_applied == case["expected_applied"]
    assert int(r.hit_round_cap) == case["expected_hit_cap"]
    if "optimum" in case:
        emap = ck.entry_map(wl.col_ptr, wl.row_idx, wl.w)
        assert float(ck.brute_force_optimum(wl.n, emap)) == case["optimum"]
        assert r.total < case["optimum"]


def test_empty_and_single():
    r = oracle_improve(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), np.zeros(0, np.int32))
    assert r.status == 0 and r.total == 0.0 and r.rounds == 0
    wl = from_dense(np.array([[-0.0]]))
    r = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, 1000)
    assert r.perm.tolist() == [0] and r.rounds == 1
    assert r.total == 0.0 and math.copysign(1.0, r.total) == -1.0


# --------------------------------------------------------------------------
# brute force, n <= 8

def _cases_small():
    out = []
    for n in range(2, 9):
        for d in (1, 2, 3, n):
            for seed in range(4):
                out.append((n, d, seed, seed % 2 == 0))
    return out


@pytest.mark.parametrize("n,d,seed,intw", _cases_small())
def test_brute_force_small(n, d, seed, intw):
    wl = small_random(n, d, 100 * n + 10 * d + seed, integer_weights=intw, weight_range=3)
    emap = ck.entry_map(wl.col_ptr, wl.row_idx, wl.w)
    r = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, max_rounds=500)
    assert r.status == 0 and not r.hit_round_cap  # the exact weight rises every round: it ends
    assert ck.is_perfect_matching(n, r.perm, emap)
    # no positive-gain 4-cycle is left at termination
    assert ck.positive_4cycles(n, r.perm, emap) == []
    # bounded by the optimum, never below the start
    opt = ck.brute_force_optimum(n, emap)
    final = ck.exact_weight(r.perm, emap)
    start = ck.exact_weight(wl.planted, emap)
    assert start <= final <= opt
    # every applied round strictly raises the exact weight and is a set of
    # vertex-disjoint positive swaps; rounds equal the one-round pair derivation
    prev = wl.planted.tolist()
    for rr in range(1, r.rounds + 1):
        step = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, prev, max_rounds=1)
        ref_perm, ref_cand, ref_app = ck.one_round_by_pairs(n, prev, emap)
        assert step.perm.tolist() == ref_perm
        assert step.round_candidates[0] == ref_cand == r.round_candidates[rr - 1]
        assert step.round_applied[0] == ref_app == r.round_applied[rr - 1]
        assert ck.round_is_disjoint_positive_swaps(n, prev, step.perm, emap)
        if ref_app:
            assert ck.exact_weight(step.perm, emap) > ck.exact_weight(prev, emap)
        prev = step.perm.tolist()
    assert prev == r.perm.tolist()
    # with integer weights, a gap to the optimum means M xor M* has a positive
    # alternating cycle, and it is longer than 4 (Section 4 optimality criterion)
    if intw and final < opt:
        best = None
        import itertools
        for p in itertools.permutations(range(n)):
            if all((p[j], j) in emap for j in range(n)):
                if sum(Fraction(emap[(p[j], j)][0]) for j in range(n)) == opt:
                    best = p
                    break
        cycles = _alt_cycles(r.perm.tolist(), list(best))
        gains = [sum(Fraction(emap[(best[j], j)][0]) - Fraction(emap[(r.perm[j], j)][0]) for j in cyc)
                 for cyc in cycles]
        assert any(g > 0 and len(cyc) >= 3 for g, cyc in zip(gains, cycles))
        assert all(not (g > 0 and len(cyc) == 2) for g, cyc in zip(gains, cycles))


def _alt_cycles(m, mstar):
    """Columns of each alternating cycle of m xor mstar (both perm arrays)."""
    n = len(m)
    col_of_row = {r: j for j, r in enumerate(m)}
    seen, out = set(), []
    for j in range(n):
        if j in seen or m[j] == mstar[j]:
            continue
        cyc, c = [], j
        while c not in seen:
            seen.add(c)
            cyc.append(c)
            c = col_of_row[mstar[c]]
        out.append(cyc)
    return out


# --------------------------------------------------------------------------
# moderate n: library optimum and invariants

@pytest.mark.parametrize("n,d,seed", [(50, 3, 1), (120, 4, 2), (300, 6, 3), (300, 2, 4)])
def test_vs_assignment_optimum(n, d, seed):
    from scipy.optimize import linear_sum_assignment
    wl = small_random(n, d, seed)
    r = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, 1000)
    assert not r.hit_round_cap
    a = ck.dense_from_workload(wl)
    cost = np.where(np.isnan(a), -1e9, a)
    rows, cols = linear_sum_assignment(cost, maximize=True)
    assert np.all(~np.isnan(a[rows, cols]))
    emap = ck.entry_map(wl.col_ptr, wl.row_idx, wl.w)
    opt = sum((Fraction(a[r_, c_]) for r_, c_ in zip(rows, cols)), Fraction(0))
    final = ck.exact_weight(r.perm, emap)
    assert final <= opt
    assert ck.positive_4cycles(n, r.perm, emap) == []


def test_equal_weights_do_nothing():
    # all weights equal: every gain is exactly 0, nothing is a candidate
    wl = small_random(200, 5, 9)
    w = np.full_like(wl.w, 0.75)
    r = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, w, wl.planted, 1000)
    assert r.rounds == 1 and r.cycles_applied == 0 and r.perm.tolist() == wl.planted.tolist()
