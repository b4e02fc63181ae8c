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

@pytest.mark.parametrize("n,d,seed,intw", [
    (1, 1, 0, False), (2, 2, 1, True), (3, 3, 2, True), (5, 2, 3, False), (8, 8, 4, True),
    (63, 3, 5, False), (64, 4, 6, True), (65, 5, 7, False), (257, 9, 8, True),
    (1000, 2, 9, False), (4099, 6, 10, True), (20011, 8, 11, False), (20011, 8, 12, True),
])
def test_random_vs_oracle(solver, n, d, seed, intw):
    wl = small_random(n, d, seed, integer_weights=intw, weight_range=2)
    run_both(solver, wl)


@pytest.mark.parametrize("tile", [4, 8, 16, 32, 64])
def test_tile_widths_identical(solver, tile):
    wl = workload(0)
    run_both(solver, wl, tile_width=tile)
    wl2 = small_random(5003, 30, 77, integer_weights=True, weight_range=1)  # heavy ties
    run_both(solver, wl2, tile_width=tile)


def test_stencil_small(solver):
    wl = stencil27(23, 17, 11, 2101, 3101, name="stencil_23x17x11")
    run_both(solver, wl)


def test_stencil_integer_ties(solver):
    wl = stencil27(16, 16, 16, 2102, 3102, name="stencil_16cubed_int")
    rng = np.random.default_rng(5)
    wl.w = rng.integers(-2, 3, size=wl.nnz).astype(np.float64)
    run_both(solver, wl)


@pytest.mark.parametrize("scale", [12, 14])
def test_rmat_long_columns(solver, scale):
    wl = rmat(scale, 16, 1000 + scale, 2000 + scale, 3000 + scale, name=f"rmat_scale{scale}")
    assert np.diff(wl.col_ptr).max() > 256  # exercises the split search
    gpu, ref = run_both(solver, wl)
    assert gpu[2]["long_columns"] > 0


def test_round_cap(solver):
    wl = stencil27(20, 20, 20, 2103, 3103, name="stencil_20cubed")
    for cap in (1, 2, 3):
        run_both(solver, wl, max_rounds=cap)


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
    for rep in range(3):
        mate = _dev(wl.planted, dev)
        res = solver.improve(cp, ri, w, mate, perm_out=mate)  # in place
        assert np.array_equal(mate.cpu().numpy(), ref.perm)
        assert res.total == ref.total


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


def test_bad_matching_rejected(solver):
    from paper_1801_09809_amd import hwpm
    wl = small_random(100, 4, 3)
    E = hwpm.HWPM_EBADMATCH
    m = wl.planted.copy(); m[3] = m[4]            # duplicate row
    _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m)
    m = wl.planted.copy(); m[3] = wl.n            # out of range
    _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m)
    m = wl.planted.copy(); m[0] = -1
    _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m)
    # a permutation that uses a structural zero
    a = ck.dense_from_workload(wl)
    for j in range(wl.n):
        for c in range(wl.n):
            if c != j and np.isnan(a[wl.planted[c], j]):
                m = wl.planted.copy(); m[j], m[c] = m[c], m[j]
                _expect(solver, E, wl.col_ptr, wl.row_idx, wl.w, m)
                return
    pytest.fail("no structural zero found")


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


def _full(solver, k, max_rounds=0):
    wl = workload(k)
    dev = solver.device
    cp, ri, w = _dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev)
    from paper_1801_09809_amd import hwpm
    assert solver.check_csc(cp, ri, w) == hwpm.HWPM_OK
    print(f"[gpu] workload {k} ({wl.name}) max_rounds={max_rounds}", flush=True)
    res = solver.improve(cp, ri, w, _dev(wl.planted, dev), max_rounds=max_rounds, check_csc=False)
    torch.cuda.synchronize()
    return wl, (res.perm.cpu().numpy(), res.total, res.stats)


@pytest.mark.parametrize("k", [1, 2])
def test_full_workload_bit_exact(solver, k):
    wl, gpu = _full(solver, k)
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    assert_same(wl, gpu, ref)
    bad, wm = _no_positive_4cycle(wl, gpu[0])
    assert bad == 0
    assert oracle_tree_sum(wm) == gpu[1]


def test_full_rmat_first_rounds_bit_exact(solver):
    wl, gpu = _full(solver, 3, max_rounds=3)
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, 3)
    assert_same(wl, gpu, ref)


def test_full_rmat_converged_properties(solver):
    wl, (perm, total, st) = _full(solver, 3)
    assert st["hit_round_cap"] == 0 and st["rounds"] > 3
    assert np.array_equal(np.sort(perm), np.arange(wl.n))
    bad, wm = _no_positive_4cycle(wl, perm)
    assert bad == 0
    assert oracle_tree_sum(wm) == total
    assert total > st["init_weight"]
    # every round with candidates flipped at least one cycle, the last none
    rc, ra = st["round_candidates"], st["round_applied"]
    assert all(a > 0 for c, a in zip(rc[:-1], ra[:-1])) and ra[-1] == 0 and rc[-1] == 0
