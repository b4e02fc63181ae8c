"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

The bar is bit-exact: the permutation, the total weight's bit pattern, the
number of rounds and the per-round candidate / applied counts must equal the
oracle's on the same seeded inputs.  Sizes span many tiles with ragged tails,
every tile width, long (split) columns, heavy ties, the degenerate cases, and
the full-size workloads in the launch configuration the benchmark times.
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle_improve, oracle_tree_sum  # noqa: E402
from tests import checkers as ck  # noqa: E402
from workloads import from_dense, random_matrix, rmat, small_random, stencil27, workload  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09809_amd import hwpm
    s = hwpm.Solver(0)
    yield s
    s.close()


def _dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def gpu_improve(solver, wl, mate=None, **kw):
    print(f"[gpu] {wl.name} n={wl.n} nnz={wl.nnz} {kw}", flush=True)
    dev = solver.device
    mate = wl.planted if mate is None else mate
    res = solver.improve(_dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev),
                         _dev(np.asarray(mate, dtype=np.int32), dev), **kw)
    torch.cuda.synchronize()
    return res.perm.cpu().numpy(), res.total, res.stats


def assert_same(wl, gpu, ref, check_init=True):
    perm, total, st = gpu
    assert np.array_equal(perm, ref.perm), f"{wl.name}: permutation differs"
    assert np.float64(total).tobytes() == np.float64(ref.total).tobytes(), \
        f"{wl.name}: total {total!r} != {ref.total!r}"
    assert st["rounds"] == ref.rounds
    assert st["hit_round_cap"] == int(ref.hit_round_cap)
    assert st["cycles_applied"] == ref.cycles_applied
    nr = min(ref.rounds, 256)
    assert st["round_candidates"][:nr] == ref.round_candidates[:nr]
    assert st["round_applied"][:nr] == ref.round_applied[:nr]
    if check_init:
        assert np.float64(st["init_weight"]).tobytes() == np.float64(ref.init_weight).tobytes()


def run_both(solver, wl, max_rounds=0, **kw):
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, max_rounds)
    gpu = gpu_improve(solver, wl, max_rounds=max_rounds, **kw)
    assert_same(wl, gpu, ref)
    return gpu, ref


# ---------------------------------------------------------------------------
# hand-derived cases

def _golden_cases():
    with open(os.path.join(GOLDEN, "wiac_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_golden_on_gpu(solver, case):
    a = np.array([[np.nan if v is None else float(v) for v in r] for r in case["dense"]])
    wl = from_dense(a, planted=case["mate_in"], name=case["name"])
    perm, total, st = gpu_improve(solver, wl, max_rounds=case["max_rounds"])
    assert perm.tolist() == case["expected_perm"]
    assert total == case["expected_total"]
    assert st["rounds"] == case["expected_rounds"]
    assert st["round_candidates"] == case["expected_candidates"]
    assert st["round_applied"] == case["expected_applied"]
    assert st["hit_round_cap"] == case["expected_hit_cap"]


# ---------------------------------------------------------------------------
# small and medium random cases, all tile widths

# search configurations: column binary search; transposed row lists; chunked
# transposed (incremental rounds, the default); chunked with full rounds
PROBES = ["p1", "p2", "p3", "p3full", "p4", "p4full", "p5", "p5full"]
_PROBE_KW = {"p1": dict(probe=1), "p2": dict(probe=2), "p3": dict(probe=3),
             "p3full": dict(probe=3, full_search=True), "p4": dict(probe=4),
             "p4full": dict(probe=4, full_search=True), "p5": dict(probe=5),
             "p5full": dict(probe=5, full_search=True)}


@pytest.mark.parametrize("probe", PROBES)
@pytest.mark.parametrize("n,d,seed,intw", [
    (1, 1, 0, False), (2, 2, 1, True), (3, 3, 2, True), (5, 2, 3, False), (8, 8, 4, True),
    (63, 3, 5, False), (64, 4, 6, True), (65, 5, 7, False), (257, 9, 8, True),
    (1000, 2, 9, False), (4099, 6, 10, True), (20011, 8, 11, False), (20011, 8, 12, True),
    (3001, 70, 13, True),  # rows longer than the rotation limit
])
def test_random_vs_oracle(solver, n, d, seed, intw, probe):
    wl = small_random(n, d, seed, integer_weights=intw, weight_range=2)
    run_both(solver, wl, **_PROBE_KW[probe])


@pytest.mark.parametrize("probe", PROBES)
@pytest.mark.parametrize("tile", [4, 8, 16, 32, 64])
def test_tile_widths_identical(solver, tile, probe):
    if probe[:2] in ("p3", "p4", "p5") and tile == 64:
        pytest.skip("the row-list tile kernels take tiles of 4 to 32 lanes")
    wl = workload(0)
    run_both(solver, wl, tile_width=tile, **_PROBE_KW[probe])
    wl2 = small_random(5003, 30, 77, integer_weights=True, weight_range=1)  # heavy ties
    run_both(solver, wl2, tile_width=tile, **_PROBE_KW[probe])


@pytest.mark.parametrize("probe", PROBES)
def test_stencil_small(solver, probe):
    wl = stencil27(23, 17, 11, 2101, 3101, name="stencil_23x17x11")
    run_both(solver, wl, **_PROBE_KW[probe])


@pytest.mark.parametrize("probe", PROBES)
def test_stencil_integer_ties(solver, probe):
    wl = stencil27(16, 16, 16, 2102, 3102, name="stencil_16cubed_int")
    rng = np.random.default_rng(5)
    wl.w = rng.integers(-2, 3, size=wl.nnz).astype(np.float64)
    run_both(solver, wl, **_PROBE_KW[probe])


@pytest.mark.parametrize("probe", PROBES)
@pytest.mark.parametrize("scale", [12, 14])
def test_rmat_long_columns(solver, scale, probe):
    wl = rmat(scale, 16, 1000 + scale, 2000 + scale, 3000 + scale, name=f"rmat_scale{scale}")
    assert np.diff(wl.col_ptr).max() > 256  # exercises the split search
    assert np.bincount(wl.row_idx).max() > 64  # and the long-row fallback
    gpu, ref = run_both(solver, wl, **_PROBE_KW[probe])
    assert gpu[2]["long_columns"] > 0


@pytest.mark.parametrize("probe", PROBES)
def test_round_cap(solver, probe):
    wl = stencil27(20, 20, 20, 2103, 3103, name="stencil_20cubed")
    for cap in (1, 2, 3):
        run_both(solver, wl, max_rounds=cap, **_PROBE_KW[probe])


def test_empty_matrix(solver):
    from paper_1801_09809_amd import hwpm
    dev = solver.device
    col_ptr = torch.zeros(1, dtype=torch.int64, device=dev)
    e_i = torch.zeros(0, dtype=torch.int32, device=dev)
    e_w = torch.zeros(0, dtype=torch.float64, device=dev)
    res = solver.improve(col_ptr, e_i, e_w, e_i)
    assert res.total == 0.0 and res.perm.numel() == 0 and res.stats["rounds"] == 0
    assert isinstance(hwpm.hwpm_strerror(0), str)


def test_single_negative_zero(solver):
    wl = from_dense(np.array([[-0.0]]), name="one_by_one")
    perm, total, st = gpu_improve(solver, wl)
    assert perm.tolist() == [0] and st["rounds"] == 1
    assert total == 0.0 and np.signbit(total)


def test_aliasing_and_determinism(solver):
    wl = small_random(30001, 7, 31)
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    dev = solver.device
    cp, ri, w = _dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev)
    for rep in range(len(PROBES)):
        mate = _dev(wl.planted, dev)
        res = solver.improve(cp, ri, w, mate, perm_out=mate, **_PROBE_KW[PROBES[rep]])  # in place
        assert np.array_equal(mate.cpu().numpy(), ref.perm)
        assert res.total == ref.total


@pytest.mark.parametrize("probe", [1, 3, 5])
def test_timing_levels(solver, probe):
    """Timing never changes the result; level 2 fills only the search-stage
    times, level 1 every stage; other levels are rejected."""
    from paper_1801_09809_amd import hwpm
    wl = small_random(20001, 9, 33)
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    by = {}
    for level in (0, 1, 2):
        gpu = gpu_improve(solver, wl, timing=level, probe=probe, full_search=True)
        assert_same(wl, gpu, ref)
        by[level] = gpu[2]
    assert by[0]["ms_search"] == 0.0 and by[0]["ms_setup"] == 0.0
    for level in (1, 2):
        st = by[level]
        assert st["ms_search"] > 0.0
        assert st["ms_search_first"] > 0.0
        assert all(x > 0.0 for x in st["round_ms_search"][:st["rounds"]])
        assert abs(sum(st["round_ms_search"][:st["rounds"]]) - st["ms_search"]) <= 1e-3 * st["ms_search"] + 1e-4
    assert by[1]["ms_setup"] > 0.0 and by[1]["ms_resolve"] > 0.0 and by[1]["ms_apply"] > 0.0
    assert by[2]["ms_setup"] == 0.0 and by[2]["ms_resolve"] == 0.0 and by[2]["ms_apply"] == 0.0
    for bad in (-1, 3):
        _expect(solver, hwpm.HWPM_EINVAL, wl.col_ptr, wl.row_idx, wl.w, wl.planted, timing=bad)


# ---------------------------------------------------------------------------
# error paths (forced from the host; the validation kernels bound every access)

def _expect(solver, status, col_ptr, row_idx, w, mate, **kw):
    from paper_1801_09809_amd import hwpm
    dev = solver.device
    with pytest.raises(hwpm.HwpmError) as e:
        solver.improve(_dev(col_ptr, dev), _dev(row_idx, dev), _dev(w, dev), _dev(mate, dev), **kw)
    assert e.value.status == status


def test_bad_csc_rejected(solver):
    from paper_1801_09809_amd import hwpm
    wl = small_random(100, 4, 3)
    E = hwpm.HWPM_EBADCSC
    ri = wl.row_idx.copy(); ri[5] = wl.n          # row out of range
    _expect(solver, E, wl.col_ptr, ri, wl.w, wl.planted)
    ri = wl.row_idx.copy(); ri[-1] = -3
    _expect(solver, E, wl.col_ptr, ri, wl.w, wl.planted)
    j = int(np.argmax(np.diff(wl.col_ptr) >= 2))  # unsorted rows inside a column
    ri = wl.row_idx.copy(); a = wl.col_ptr[j]; ri[a], ri[a + 1] = ri[a + 1], ri[a]
    _expect(solver, E, wl.col_ptr, ri, wl.w, wl.planted)
    ri = wl.row_idx.copy(); ri[a + 1] = ri[a]     # duplicate row
    _expect(solver, E, wl.col_ptr, ri, wl.w, wl.planted)
    for bad in (np.nan, np.inf, -np.inf):
        w = wl.w.copy(); w[7] = bad
        _expect(solver, E, wl.col_ptr, wl.row_idx, w, wl.planted)
    cp = wl.col_ptr.copy(); cp[10], cp[11] = cp[11], cp[10]   # decreasing
    if cp[10] != cp[11]:
        _expect(solver, E, cp, wl.row_idx, wl.w, wl.planted)
    cp = wl.col_ptr.copy(); cp[0] = 1
    _expect(solver, E, cp, wl.row_idx, wl.w, wl.planted)
    cp = wl.col_ptr.copy(); cp[-1] = wl.nnz - 1
    _expect(solver, E, cp, wl.row_idx, wl.w, wl.planted)
    cp = wl.col_ptr.copy(); cp[50] = 1 << 40
    _expect(solver, E, cp, wl.row_idx, wl.w, wl.planted)
    # the standalone check agrees
    dev = solver.device
    assert solver.check_csc(_dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev)) == hwpm.HWPM_OK
    ri = wl.row_idx.copy(); ri[5] = wl.n
    assert solver.check_csc(_dev(wl.col_ptr, dev), _dev(ri, dev), _dev(wl.w, dev)) == E


@pytest.mark.parametrize("probe", [1, 2, 3, 4, 5])
def test_bad_matching_rejected(solver, probe):
    from paper_1801_09809_amd import hwpm
    wl = small_random(100, 4, 3)
    E = hwpm.HWPM_EBADMATCH
    m = wl.planted.copy(); m[3] = m[4]            # duplicate row
    _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m, probe=probe)
    m = wl.planted.copy(); m[3] = wl.n            # out of range
    _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m, probe=probe)
    m = wl.planted.copy(); m[0] = -1
    _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m, probe=probe)
    # a permutation that uses a structural zero
    a = ck.dense_from_workload(wl)
    for j in range(wl.n):
        for c in range(wl.n):
            if c != j and np.isnan(a[wl.planted[c], j]):
                m = wl.planted.copy(); m[j], m[c] = m[c], m[j]
                _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m, probe=probe)
                return
    pytest.fail("no structural zero found")


@pytest.mark.parametrize("probe", [1, 3, 5])
def test_structural_zero_matching_leaves_outputs(solver, probe):
    """A permutation with one mate row outside its column, on a matrix of many
    transpose tiles: HWPM_EBADMATCH before any round, the output untouched,
    and a valid solve on the same handle right after gives the oracle's
    result."""
    from paper_1801_09809_amd import hwpm
    dev = solver.device
    wl = small_random(20000, 8, 17)
    col0 = set(wl.row_idx[wl.col_ptr[0]:wl.col_ptr[1]].tolist())
    c = next(c for c in range(1, wl.n) if int(wl.planted[c]) not in col0)
    m = wl.planted.copy(); m[0], m[c] = m[c], m[0]
    cp, ri, w = _dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev)
    perm = torch.full((wl.n,), -7, dtype=torch.int32, device=dev)
    print(f"[gpu] structural zero n={wl.n} probe={probe} column 0 <-> {c}", flush=True)
    with pytest.raises(hwpm.HwpmError) as e:
        solver.improve(cp, ri, w, _dev(m, dev), perm_out=perm, probe=probe)
    assert e.value.status == hwpm.HWPM_EBADMATCH
    assert bool((perm == -7).all())
    res = solver.improve(cp, ri, w, _dev(wl.planted, dev), perm_out=perm, probe=probe)
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    assert np.array_equal(perm.cpu().numpy(), ref.perm)
    assert np.float64(res.total).tobytes() == np.float64(ref.total).tobytes()
    assert np.float64(res.stats["init_weight"]).tobytes() == np.float64(ref.init_weight).tobytes()


@pytest.mark.parametrize("probe", [1, 2, 3, 4, 5])
def test_matching_without_entries(solver, probe):
    """n > 0 columns and no entries: no perfect matching lies in the
    pattern, whatever permutation is given (refused on the host, before any
    kernel reads the empty entry arrays)."""
    from paper_1801_09809_amd import hwpm
    n = 7
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    ri, w = np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.float64)
    mate = np.arange(n, dtype=np.int32)
    _expect(solver, hwpm.HWPM_EBADMATCH, col_ptr, ri, w, mate, probe=probe)
    _expect(solver, hwpm.HWPM_EBADMATCH, col_ptr, ri, w, mate, probe=probe, check_csc=False)


# ---------------------------------------------------------------------------
# full-size workloads, in the configuration the benchmark times
# (CSC validated once, then tile 16, check_csc = 0)

def _no_positive_4cycle(wl, perm):
    """Vectorised termination check: no column j, row i > m_j of j, with the
    closing edge {m_j, m_i} present and a positive grouped gain."""
    n = wl.n
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(wl.col_ptr))
    rows = wl.row_idx.astype(np.int64)
    key = cols * n + rows
    mc = perm.astype(np.int64)
    mr = np.empty(n, dtype=np.int64); mr[mc] = np.arange(n)
    pos_m = np.searchsorted(key, np.arange(n, dtype=np.int64) * n + mc)
    assert np.array_equal(key[pos_m], np.arange(n) * n + mc), "matching leaves the pattern"
    wm = wl.w[pos_m]
    sel = np.nonzero(rows > mc[cols])[0]
    i, j = rows[sel], cols[sel]
    mi, mj = mr[i], mc[j]
    q = mi * n + mj
    p = np.searchsorted(key, q)
    p[p >= key.size] = 0
    hit = key[p] == q
    g = (wl.w[sel[hit]] + wl.w[p[hit]]) - (wm[mi[hit]] + wm[j[hit]])
    return int((g > 0).sum()), wm


def _full(solver, k, max_rounds=0, probe="p3"):
    wl = workload(k)
    dev = solver.device
    cp, ri, w = _dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev)
    from paper_1801_09809_amd import hwpm
    assert solver.check_csc(cp, ri, w) == hwpm.HWPM_OK
    print(f"[gpu] workload {k} ({wl.name}) max_rounds={max_rounds} probe={probe}", flush=True)
    res = solver.improve(cp, ri, w, _dev(wl.planted, dev), max_rounds=max_rounds, check_csc=False,
                         **_PROBE_KW[probe])
    torch.cuda.synchronize()
    return wl, (res.perm.cpu().numpy(), res.total, res.stats)


@pytest.mark.parametrize("k", [1, 2])
def test_full_workload_bit_exact(solver, k):
    wl, gpu = _full(solver, k, probe="p3full")  # the benchmark's configuration
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    assert_same(wl, gpu, ref)
    bad, wm = _no_positive_4cycle(wl, gpu[0])
    assert bad == 0
    assert oracle_tree_sum(wm) == gpu[1]
    for probe in PROBES:
        _, other = _full(solver, k, probe=probe)
        assert_same(wl, other, ref)


@pytest.mark.parametrize("probe", PROBES)
def test_full_rmat_first_rounds_bit_exact(solver, probe):
    wl, gpu = _full(solver, 3, max_rounds=3, probe=probe)
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, 3)
    assert_same(wl, gpu, ref)


def _golden_rmat():
    with open(os.path.join(GOLDEN, "rmat_scale22_converged.json")) as f:
        return json.load(f)


def _digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _first_round_diff(got, want):
    for r, (g, w) in enumerate(zip(got, want)):
        if g != w:
            return r
    return None if len(got) == len(want) else min(len(got), len(want))


@pytest.mark.parametrize("probe,cap", [("p3", 0), ("p3full", 0), ("p5", 0), ("p4", 0), ("p3", 10)])
def test_full_rmat_vs_oracle_golden(solver, probe, cap):
    """R-MAT scale 22 solved from its planted matching (119 rounds to
    convergence, and the paper's cap of 10) against the oracle's stored
    result (tests/golden/make_rmat_golden.py runs the oracle alone): the
    permutation's digest, the totals' bit patterns and every round's
    candidate and flip counts."""
    gold = _golden_rmat()
    wl, (perm, total, st) = _full(solver, 3, max_rounds=cap, probe=probe)
    assert (wl.n, wl.nnz) == (gold["n"], gold["nnz"])
    for name, arr in (("col_ptr", wl.col_ptr), ("row_idx", wl.row_idx), ("w", wl.w), ("planted", wl.planted)):
        assert _digest(arr) == gold["input_sha256"][name], f"regenerated {name} differs from the recorded input"
    ref = gold["converged" if cap == 0 else "maxiters_10"]
    rounds = ref["rounds"]
    cand, flips = st["round_candidates"][:rounds], st["round_applied"][:rounds]
    r = _first_round_diff(cand, ref["round_candidates"])
    assert r is None, f"round {r}: {cand[r] if r < len(cand) else None} candidates, oracle {ref['round_candidates'][r]}"
    r = _first_round_diff(flips, ref["round_applied"])
    assert r is None, f"round {r}: {flips[r] if r < len(flips) else None} flips, oracle {ref['round_applied'][r]}"
    assert st["rounds"] == rounds and st["hit_round_cap"] == int(ref["hit_round_cap"])
    assert st["cycles_applied"] == ref["cycles_applied"]
    assert np.float64(st["init_weight"]).tobytes()[::-1].hex() == ref["init_weight_bits"]
    assert np.float64(total).tobytes()[::-1].hex() == ref["total_bits"]
    assert _digest(perm.astype(np.int32)) == ref["perm_sha256"]


def test_full_rmat_converged_properties(solver):
    wl, (perm, total, st) = _full(solver, 3, probe="p3")  # default: incremental rounds
    _, other = _full(solver, 3, probe="p3full")
    assert np.array_equal(other[0], perm) and other[1] == total
    assert other[2]["round_applied"] == st["round_applied"]
    assert st["hit_round_cap"] == 0 and st["rounds"] > 3
    _, light = _full(solver, 3, probe="p5")  # lists without positions: searched mate refreshes
    assert np.array_equal(light[0], perm) and light[1] == total
    assert light[2]["round_applied"] == st["round_applied"]
    assert np.array_equal(np.sort(perm), np.arange(wl.n))
    bad, wm = _no_positive_4cycle(wl, perm)
    assert bad == 0
    assert oracle_tree_sum(wm) == total
    assert total > st["init_weight"]
    # every round with candidates flipped at least one cycle, the last none
    rc, ra = st["round_candidates"], st["round_applied"]
    assert all(a > 0 for c, a in zip(rc[:-1], ra[:-1])) and ra[-1] == 0 and rc[-1] == 0


# ---------------------------------------------------------------------------
# the whole pipeline (greedy + BFS matching + rounds) against the oracle

def gpu_match(solver, wl, **kw):
    print(f"[gpu] match {wl.name} n={wl.n} nnz={wl.nnz} {kw}", flush=True)
    dev = solver.device
    res = solver.match(_dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev), **kw)
    torch.cuda.synchronize()
    return res.perm.cpu().numpy(), res.total, res.stats


def match_both(solver, wl, plain=False, **kw):
    from oracle import oracle_greedy, oracle_match
    ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w, heavy=not plain,
                       max_rounds=kw.get("max_rounds", 0))
    gcard, _, _ = oracle_greedy(wl.n, wl.col_ptr, wl.row_idx, wl.w, heavy=not plain)
    gpu = gpu_match(solver, wl, mcm_plain=plain, **kw)
    assert_same(wl, gpu, ref)
    st = gpu[2]
    assert st["greedy_cardinality"] == gcard == ref.greedy_cardinality
    assert st["mcm_cardinality"] == ref.mcm_cardinality == wl.n
    # Phase I step counts: proposal rounds, BFS phases and levels
    assert (st["greedy_rounds"], st["mcm_phases"], st["mcm_levels"]) == \
        (ref.greedy_rounds, ref.mcm_phases, ref.mcm_levels)
    return gpu, ref


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("n,d,seed,intw", [
    (1, 1, 0, False), (2, 1, 1, True), (7, 2, 2, True), (64, 1, 3, False), (65, 2, 4, True),
    (1000, 1, 5, False), (3001, 3, 6, True), (20011, 2, 7, False), (20011, 6, 8, True),
])
def test_match_random_vs_oracle(solver, n, d, seed, intw, plain):
    wl = small_random(n, d, seed, integer_weights=intw, weight_range=2)
    match_both(solver, wl, plain=plain)


@pytest.mark.parametrize("plain", [False, True])
def test_match_stencil_and_rmat(solver, plain):
    match_both(solver, stencil27(21, 13, 9, 2104, 3104, name="stencil_21x13x9"), plain=plain)
    match_both(solver, rmat(13, 16, 1013, 2013, 3013, name="rmat_scale13"), plain=plain)


def test_match_singular(solver):
    from paper_1801_09809_amd import hwpm
    from oracle import oracle_match
    dev = solver.device
    for n, holes, seed in ((50, 0.3, 1), (2000, 0.2, 2), (5000, 0.05, 3)):
        wl = small_random(n, 1, seed)
        rng = np.random.default_rng(seed)
        keep = np.ones(wl.nnz, dtype=bool)
        for j in range(n):  # drop planted entries so the matrix may be singular
            if rng.random() < holes:
                lo, hi = wl.col_ptr[j], wl.col_ptr[j + 1]
                keep[lo + np.searchsorted(wl.row_idx[lo:hi], wl.planted[j])] = False
        counts = np.array([keep[wl.col_ptr[j]:wl.col_ptr[j + 1]].sum() for j in range(n)])
        cp = np.zeros(n + 1, dtype=np.int64); cp[1:] = np.cumsum(counts)
        ri, w = wl.row_idx[keep], wl.w[keep]
        ref = oracle_match(n, cp, ri, w)
        perm = torch.full((n,), -7, dtype=torch.int32, device=dev)
        if ref.status == -2:
            with pytest.raises(hwpm.HwpmError) as e:
                solver.match(_dev(cp, dev), _dev(ri, dev), _dev(w, dev), perm_out=perm)
            assert e.value.status == hwpm.HWPM_ESINGULAR
            assert (perm.cpu().numpy() == -7).all()  # outputs untouched
        else:
            res = solver.match(_dev(cp, dev), _dev(ri, dev), _dev(w, dev), perm_out=perm)
            assert np.array_equal(perm.cpu().numpy(), ref.perm) and res.total == ref.total


def test_match_fewer_entries_than_columns(solver):
    """No perfect matching fits in fewer than n entries: HWPM_ESINGULAR (as
    the oracle finds), refused on the host, the output untouched."""
    from paper_1801_09809_amd import hwpm
    from oracle import oracle_match
    dev = solver.device
    cases = [(np.zeros(7, dtype=np.int64), np.zeros(0, dtype=np.int32)),       # n = 6, no entries
             (np.array([0, 1, 2, 3, 3], dtype=np.int64), np.array([2, 0, 1], dtype=np.int32))]  # n = 4, 3 entries
    for cp, ri in cases:
        n = cp.size - 1
        w = np.linspace(1.0, 2.0, ri.size)
        assert oracle_match(n, cp, ri, w).status == -2
        for check in (True, False):
            perm = torch.full((n,), -7, dtype=torch.int32, device=dev)
            with pytest.raises(hwpm.HwpmError) as e:
                solver.match(_dev(cp, dev), _dev(ri, dev), _dev(w, dev), perm_out=perm, check_csc=check)
            assert e.value.status == hwpm.HWPM_ESINGULAR
            assert (perm.cpu().numpy() == -7).all()


@pytest.mark.parametrize("k", [1, 2])
def test_match_full_workload(solver, k):
    wl = workload(k)
    match_both(solver, wl, check_csc=True)


# ---------------------------------------------------------------------------
# the paper's variants on the same kernels

def test_variant_option_a_objective(solver):
    """Sum of |a| instead of sum of log|a| (Option A): only the weights change."""
    from workloads import option_a
    for wl in (option_a(small_random(20011, 8, 41)), option_a(stencil27(19, 17, 13, 2105, 3105))):
        run_both(solver, wl)
        match_both(solver, wl)


def test_variant_maxiters_10(solver):
    """The paper's cap of 10 rounds, on an R-MAT matrix that needs more."""
    wl = rmat(14, 16, 1014, 2014, 3014, name="rmat_scale14")
    gpu, ref = run_both(solver, wl, max_rounds=10)
    assert ref.hit_round_cap and gpu[2]["hit_round_cap"] == 1 and gpu[2]["rounds"] == 10
    run_both(solver, wl, max_rounds=10, probe=1)


@pytest.mark.parametrize("plain", [False, True])
def test_variant_equilibrated_ties(solver, plain):
    """Equilibrated matrices: the largest entry of every row and column has
    weight exactly 0, so equal gains and equal proposal weights are common."""
    from workloads import equilibrated
    for wl in (equilibrated(small_random(30011, 6, 43)), equilibrated(stencil27(21, 21, 11, 2106, 3106))):
        assert (wl.w == 0.0).sum() > wl.n // 2
        if not plain:
            run_both(solver, wl)
            run_both(solver, wl, probe=1)
        match_both(solver, wl, plain=plain)


# ---------------------------------------------------------------------------
# batches: every matrix gets exactly its own result

def _mixed_batch(seed, count=9):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        kind = b % 3
        if kind == 0:
            out.append(small_random(int(rng.integers(1, 3000)), int(rng.integers(1, 9)), seed * 100 + b,
                                    integer_weights=bool(b % 2), weight_range=2))
        elif kind == 1:
            g = int(rng.integers(3, 14))
            out.append(stencil27(g, g, g, seed * 100 + b, seed * 200 + b, n_keep=int(rng.integers(1, g ** 3 + 1))))
        else:
            out.append(rmat(int(rng.integers(6, 11)), 8, seed + b, seed + 2 * b, seed + 3 * b,
                            name=f"rmat_small{b}"))
    return out


@pytest.mark.parametrize("probe", ["p1", "p3", "p4", "p5"])
def test_improve_batch_equals_alone(solver, probe):
    from oracle import oracle_improve
    dev = solver.device
    # an empty member runs no search pass (rounds 0), as alone
    wls = _mixed_batch(5) + [small_random(1, 1, 3), small_random(0, 1, 1), workload(0)]
    mats = [(_dev(w.col_ptr, dev), _dev(w.row_idx, dev), _dev(w.w, dev)) for w in wls]
    mates = [_dev(w.planted, dev) for w in wls]
    perms, totals, items, bst = solver.improve_batch(mats, mates, **_PROBE_KW[probe])
    for wl, p, t, it in zip(wls, perms, totals, items):
        ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
        assert np.array_equal(p.cpu().numpy(), ref.perm), wl.name
        assert np.float64(t).tobytes() == np.float64(ref.total).tobytes()
        assert it["rounds"] == ref.rounds and it["cycles_applied"] == ref.cycles_applied
        assert np.float64(it["init_weight"]).tobytes() == np.float64(ref.init_weight).tobytes()
    assert bst["rounds"] == max(it["rounds"] for it in items)
    # with a cap
    perms, totals, items, _ = solver.improve_batch(mats, mates, max_rounds=2, **_PROBE_KW[probe])
    for wl, p, t, it in zip(wls, perms, totals, items):
        ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, 2)
        assert np.array_equal(p.cpu().numpy(), ref.perm) and t == ref.total
        assert it["rounds"] == ref.rounds and it["hit_round_cap"] == int(ref.hit_round_cap)


@pytest.mark.parametrize("plain", [False, True])
def test_match_batch_equals_alone_with_singular(solver, plain):
    from oracle import oracle_match
    dev = solver.device
    wls = _mixed_batch(7)
    # a structurally singular member: its last row is empty
    nan = np.nan
    wls.insert(3, from_dense(np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [nan, nan, nan]]),
                             name="singular3"))
    mats = [(_dev(w.col_ptr, dev), _dev(w.row_idx, dev), _dev(w.w, dev)) for w in wls]
    perms = [torch.full((w.n,), -7, dtype=torch.int32, device=dev) for w in wls]
    perms, totals, items, _ = solver.match_batch(mats, perms=perms, mcm_plain=plain)
    for wl, p, t, it in zip(wls, perms, totals, items):
        ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w, heavy=not plain)
        if ref.status == -2:
            assert it["status"] == -2 and (p.cpu().numpy() == -7).all(), wl.name
            continue
        assert it["status"] == 0
        assert np.array_equal(p.cpu().numpy(), ref.perm), wl.name
        assert np.float64(t).tobytes() == np.float64(ref.total).tobytes()
        assert it["rounds"] == ref.rounds


def test_batch_members_without_entries(solver):
    """A member with columns but no entries: hwpm_match_batch reports it
    singular (as the oracle does) and solves the others; hwpm_improve_batch
    rejects the batch's matching; a batch of such members only is all
    singular."""
    from paper_1801_09809_amd import hwpm
    from oracle import oracle_match
    dev = solver.device
    empty5 = (np.zeros(6, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.float64))
    empty3 = (np.zeros(4, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.float64))
    good = [small_random(300, 3, 1), small_random(200, 3, 2)]
    host = [(good[0].col_ptr, good[0].row_idx, good[0].w), empty5, (good[1].col_ptr, good[1].row_idx, good[1].w)]
    mats = [tuple(_dev(a, dev) for a in m) for m in host]
    perms = [torch.full((m[0].size - 1,), -7, dtype=torch.int32, device=dev) for m in host]
    print("[gpu] batch with an entry-less member", flush=True)
    perms, totals, items, _ = solver.match_batch(mats, perms=perms)
    for (cp, ri, w), p, t, it in zip(host, perms, totals, items):
        ref = oracle_match(cp.size - 1, cp, ri, w)
        if ref.status == -2:
            assert it["status"] == -2 and (p.cpu().numpy() == -7).all()
            continue
        assert it["status"] == 0 and np.array_equal(p.cpu().numpy(), ref.perm)
        assert np.float64(t).tobytes() == np.float64(ref.total).tobytes()
    assert [it["status"] for it in items] == [0, -2, 0]
    mates = [_dev(good[0].planted, dev), _dev(np.arange(5, dtype=np.int32), dev), _dev(good[1].planted, dev)]
    with pytest.raises(hwpm.HwpmError) as e:
        solver.improve_batch(mats, mates)
    assert e.value.status == hwpm.HWPM_EBADMATCH
    print("[gpu] batch of entry-less members only", flush=True)
    mats = [tuple(_dev(a, dev) for a in m) for m in (empty5, empty3)]
    perms, totals, items, _ = solver.match_batch(mats)
    assert [it["status"] for it in items] == [-2, -2]


def test_batch_rejects_bad_member(solver):
    from paper_1801_09809_amd import hwpm
    dev = solver.device
    good, bad = small_random(300, 3, 1), small_random(200, 3, 2)
    ri = bad.row_idx.copy(); ri[10] = 250  # inside the packed range, outside its block
    mats = [(_dev(good.col_ptr, dev), _dev(good.row_idx, dev), _dev(good.w, dev)),
            (_dev(bad.col_ptr, dev), _dev(ri, dev), _dev(bad.w, dev))]
    mates = [_dev(good.planted, dev), _dev(bad.planted, dev)]
    with pytest.raises(hwpm.HwpmError) as e:
        solver.improve_batch(mats, mates, check_csc=False)
    assert e.value.status == hwpm.HWPM_EBADCSC
    m2 = bad.planted.copy(); m2[0] = 200
    mats[1] = (_dev(bad.col_ptr, dev), _dev(bad.row_idx, dev), _dev(bad.w, dev))
    with pytest.raises(hwpm.HwpmError) as e:
        solver.improve_batch(mats, [mates[0], _dev(m2, dev)])
    assert e.value.status == hwpm.HWPM_EBADMATCH
    perms, totals, items, _ = solver.improve_batch([], [])
    assert perms == [] and totals == []


# ---------------------------------------------------------------------------
# launch-configuration tuner: picks a configuration, never changes a result

@pytest.mark.parametrize("which", ["random", "rmat"])
def test_autotune_keeps_the_result(solver, which):
    from paper_1801_09809_amd import hwpm
    wl = small_random(30000, 12, 77) if which == "random" else rmat(12, 16, 1012, 2012, 3012, name="rmat_s12")
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    dev = solver.device
    print(f"[gpu] autotune {wl.name} n={wl.n} nnz={wl.nnz}", flush=True)
    probe, tile, ms, perm = solver.autotune(_dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev),
                                            _dev(wl.planted, dev))
    assert (probe, tile) in hwpm.TUNE_CONFIGS
    assert all(0.0 < v < 1e30 for v in ms.values())
    assert min(ms, key=ms.get) == (probe, tile)
    assert np.array_equal(perm.cpu().numpy(), ref.perm)
    assert_same(wl, gpu_improve(solver, wl, probe=probe, tile_width=tile), ref)


# ---------------------------------------------------------------------------
# replayed graphs: batches of launches that repeat (8 rounds from the same
# ring slot, 8 proposal rounds, 8 BFS levels) are captured once per call and
# replayed; the results equal direct launches and the oracle bit for bit

def _chain(n):
    """Bidiagonal matrix whose heavier subdiagonal makes the greedy step leave
    one augmenting path through every column (one BFS phase of n levels)."""
    nan = np.nan
    a = np.full((n, n), nan)
    for j in range(n):
        a[j, j] = 1.0
        if j + 1 < n:
            a[j + 1, j] = 2.0
    return from_dense(a, name=f"chain{n}")


def _ordered(n):
    """Dense matrix whose rows are heavier the smaller their index: every
    greedy round matches one row (n proposal rounds)."""
    a = np.tile(-np.arange(n, dtype=np.float64)[:, None], (1, n))
    return from_dense(a, name=f"ordered{n}")


@pytest.mark.parametrize("case", ["rmat14", "stencil", "chain", "ordered"])
def test_graph_replay_identical(solver, case):
    from oracle import oracle_match
    wl = {"rmat14": lambda: rmat(14, 16, 1014, 2014, 3014, name="rmat_scale14"),
          "stencil": lambda: stencil27(24, 24, 24, 2107, 3107, name="stencil_24cubed"),
          "chain": lambda: _chain(61),
          "ordered": lambda: _ordered(40)}[case]()
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    for probe in ("p3", "p5"):
        runs = [gpu_improve(solver, wl, graph=g, **_PROBE_KW[probe]) for g in (True, False, True)]
        for gpu in runs:
            assert_same(wl, gpu, ref)
        if ref.rounds > 6:  # rounds 6..13 form the first replayable batch
            assert runs[0][2]["graph_launches"] > 0 and runs[1][2]["graph_launches"] == 0
    mref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w)
    for g in (True, False):
        gpu = gpu_match(solver, wl, graph=g)
        assert_same(wl, gpu, mref)
        assert (gpu[2]["greedy_rounds"], gpu[2]["mcm_phases"], gpu[2]["mcm_levels"]) == \
            (mref.greedy_rounds, mref.mcm_phases, mref.mcm_levels)
        if g and (mref.greedy_rounds > 7 or mref.mcm_levels > 7 or mref.rounds > 6):
            assert gpu[2]["graph_launches"] > 0
        if not g:
            assert gpu[2]["graph_launches"] == 0


def test_graph_replay_in_batches(solver):
    from oracle import oracle_match
    dev = solver.device
    wls = [rmat(12, 16, 1012, 2012, 3012, name="rmat_s12"), _chain(61), _ordered(40),
           small_random(3000, 5, 61)]
    mats = [(_dev(w.col_ptr, dev), _dev(w.row_idx, dev), _dev(w.w, dev)) for w in wls]
    outs = []
    for g in (True, False):
        perms, totals, items, bst = solver.match_batch(mats, graph=g)
        outs.append(([p.cpu().numpy() for p in perms], totals, bst))
        if not g:
            assert bst["graph_launches"] == 0
    for b, wl in enumerate(wls):
        ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w)
        for perms, totals, _ in outs:
            assert np.array_equal(perms[b], ref.perm), wl.name
            assert np.float64(totals[b]).tobytes() == np.float64(ref.total).tobytes()


# ---------------------------------------------------------------------------
# tuning table by degree bin: batches with default launch options take their
# bin's tuned configuration; results never change

def test_tune_table_in_batches(solver):
    from paper_1801_09809_amd import hwpm
    from oracle import oracle_match
    dev = solver.device
    sparse, dense = small_random(30000, 8, 71), stencil27(20, 20, 20, 2108, 3108, name="stencil_20cubed")
    table = None
    for wl in (sparse, dense):
        print(f"[gpu] tune bin of {wl.name}", flush=True)
        table = solver.autotune_table(_dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev),
                                      _dev(wl.planted, dev), table)
    bins = {hwpm.hwpm_tune_bin(table, wl.n, wl.nnz) for wl in (sparse, dense)}
    assert len(bins) == 2 and all(table.probe[b] != 0 for b in bins)
    solver.set_tune_table(table)
    try:
        for members in ([sparse], [dense], [dense, small_random(500, 20, 72)]):
            n_tot = sum(w.n for w in members)
            nnz_tot = sum(w.nnz for w in members)
            b = hwpm.hwpm_tune_bin(table, n_tot, nnz_tot)
            mats = [(_dev(w.col_ptr, dev), _dev(w.row_idx, dev), _dev(w.w, dev)) for w in members]
            perms, totals, items, bst = solver.match_batch(mats)
            if table.probe[b] != 0:
                assert (bst["probe_used"], bst["tile_used"]) == (table.probe[b], table.tile_width[b])
            for wl, p, t in zip(members, perms, totals):
                ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w)
                assert np.array_equal(p.cpu().numpy(), ref.perm) and t == ref.total, wl.name
    finally:
        solver.set_tune_table(None)
