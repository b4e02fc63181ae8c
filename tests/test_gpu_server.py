"""GPU tests of the serving form (hwpm_submit / hwpm_poll): every served
result equals the oracle's hwpm_match result for that matrix alone, bit for
bit, however the requests were batched, admitted or spread over workers."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle_match  # noqa: E402
from workloads import from_dense, rmat, small_random, stencil27  # noqa: E402

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09809_amd import hwpm
    return hwpm


def _requests(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        kind = b % 4
        if kind == 0:
            out.append(small_random(int(rng.integers(1, 2500)), int(rng.integers(1, 7)), seed * 1000 + b,
                                    integer_weights=bool(b % 3 == 0), weight_range=2))
        elif kind == 1:
            g = int(rng.integers(3, 12))
            out.append(stencil27(g, g, g, seed * 1000 + b, seed * 2000 + b,
                                 n_keep=int(rng.integers(1, g ** 3 + 1))))
        elif kind == 2:
            out.append(rmat(int(rng.integers(5, 10)), 8, seed + b, seed + 2 * b, seed + 3 * b,
                            name=f"rmat_srv{b}"))
        else:
            out.append(small_random(int(rng.integers(1, 40)), 2, seed * 1000 + b))
    return out


def _check(wl, res, plain=False):
    st, perm, total, info = res
    ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w, heavy=not plain)
    if ref.status == -2:
        assert st == -2 and perm is None, wl.name
        return
    assert st == 0, (wl.name, st)
    assert np.array_equal(perm, ref.perm), wl.name
    assert np.float64(total).tobytes() == np.float64(ref.total).tobytes(), wl.name
    assert info["rounds"] == ref.rounds and info["cycles_applied"] == ref.cycles_applied
    assert info["latency_ms"] >= info["queue_ms"] >= 0.0
    assert info["batch_size"] >= 1


@pytest.mark.parametrize("workers,max_batch", [(1, 64), (2, 64), (4, 8), (1, 1)])
def test_served_equals_oracle(workers, max_batch):
    hwpm = _need_gpu()
    wls = _requests(11 + workers, 24)
    nan = np.nan
    wls.insert(5, from_dense(np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [nan, nan, nan]]),
                             name="singular3"))
    wls.insert(9, small_random(0, 1, 1))
    print(f"[gpu] server workers={workers} max_batch={max_batch} requests={len(wls)}", flush=True)
    with hwpm.Server(workers=workers, max_batch=max_batch, arena_bytes=256 << 20) as srv:
        tickets = [srv.submit(w.col_ptr, w.row_idx, w.w) for w in wls]
        results = [srv.poll(t) for t in tickets]
        stats = srv.stats()
    for wl, res in zip(wls, results):
        _check(wl, res)
    assert stats["submitted"] == stats["completed"] == len(wls)
    assert stats["pending"] == 0 and stats["running"] == 0 and stats["arena_in_use"] == 0
    assert stats["max_batch_seen"] <= max_batch
    assert 0 < stats["arena_peak"] <= 256 << 20
    if max_batch == 1:
        # one request per step; a request whose rounds outlast a step takes more
        assert stats["batches"] >= len(wls) and stats["joined"] == 0


def test_continuous_batching_admits_waiting_requests():
    """With one worker, requests that arrive while a batch runs are packed
    into the next batch (their footprint permitting)."""
    hwpm = _need_gpu()
    big = stencil27(40, 40, 40, 7, 8, name="stencil_40cubed")
    small = _requests(3, 30)
    with hwpm.Server(workers=1, max_batch=64, arena_bytes=1 << 30) as srv:
        t0 = srv.submit(big.col_ptr, big.row_idx, big.w)
        ts = [srv.submit(w.col_ptr, w.row_idx, w.w) for w in small]
        results = [srv.poll(t) for t in [t0] + ts]
        stats = srv.stats()
    for wl, res in zip([big] + small, results):
        _check(wl, res)
    assert stats["batches"] < 1 + len(small)
    assert stats["max_batch_seen"] > 1


def test_requests_join_rounds_in_flight():
    """With one worker and one round per step, requests that arrive while a
    request's rounds run join its next round batch (packed with it); every
    result -- permutation, total, round and cycle counts -- still equals the
    oracle's for the matrix alone, and the long request took one step per
    round."""
    hwpm = _need_gpu()
    big = stencil27(24, 24, 24, 35, 45, name="stencil_24cubed")
    ref_big = oracle_match(big.n, big.col_ptr, big.row_idx, big.w)
    assert ref_big.rounds >= 3
    small = _requests(17, 16)
    print(f"[gpu] joining: {big.name} ({ref_big.rounds} rounds) + {len(small)} requests", flush=True)
    with hwpm.Server(workers=1, max_batch=64, arena_bytes=1 << 30, rounds_per_step=1) as srv:
        t0 = srv.submit(big.col_ptr, big.row_idx, big.w)
        deadline = time.time() + 60
        while srv.stats()["running"] == 0 and time.time() < deadline:
            time.sleep(0.0002)
        ts = [srv.submit(w.col_ptr, w.row_idx, w.w) for w in small]
        results = [srv.poll(t) for t in [t0] + ts]
        stats = srv.stats()
    for wl, res in zip([big] + small, results):
        _check(wl, res)
    assert results[0][3]["steps"] == ref_big.rounds
    assert stats["joined"] > 0
    assert stats["pending"] == 0 and stats["running"] == 0 and stats["arena_in_use"] == 0


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_round_cap_over_steps(cap):
    """solve.max_rounds caps each request's own rounds over all its steps:
    rounds, hit_round_cap and the result equal the oracle's with that cap."""
    hwpm = _need_gpu()
    wls = [stencil27(16, 16, 16, 3, 4, name="stencil_16cubed"), small_random(3000, 6, 12),
           rmat(10, 16, 1010, 2010, 3010, name="rmat_s10"), small_random(0, 1, 1)]
    with hwpm.Server(workers=1, max_batch=64, arena_bytes=256 << 20, rounds_per_step=2, max_rounds=cap) as srv:
        results = [srv.poll(t) for t in [srv.submit(w.col_ptr, w.row_idx, w.w) for w in wls]]
    for wl, (st, perm, total, info) in zip(wls, results):
        ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w, max_rounds=cap)
        assert st == 0 and ref.status == 0, wl.name
        assert np.array_equal(perm[:wl.n], ref.perm), wl.name
        assert np.float64(total).tobytes() == np.float64(ref.total).tobytes(), wl.name
        assert (info["rounds"], bool(info["hit_round_cap"]), info["cycles_applied"]) == \
            (ref.rounds, bool(ref.hit_round_cap), ref.cycles_applied), wl.name
        assert np.float64(info["init_weight"]).tobytes() == np.float64(ref.init_weight).tobytes(), wl.name


def test_submit_copies_inputs():
    """By default hwpm_submit copies the host arrays: the caller may overwrite
    them at once; with copy_inputs off they are read later (and kept alive by
    the binding until polled)."""
    hwpm = _need_gpu()
    wl = small_random(2000, 5, 77)
    for copy in (True, False):
        with hwpm.Server(workers=1, copy_inputs=copy) as srv:
            cp, ri, w = wl.col_ptr.copy(), wl.row_idx.copy(), wl.w.copy()
            t = srv.submit(cp, ri, w)
            if copy:
                cp[1:] = 0
                ri[:] = 0
                w[:] = np.nan
            res = srv.poll(t)
        _check(wl, res)


def test_admission_by_footprint():
    """An arena that holds about one request at a time still serves them all,
    one batch each; a request larger than the arena fails alone."""
    hwpm = _need_gpu()
    from paper_1801_09809_amd.hwpm import hwpm_batch_workspace_bytes
    wls = [small_random(3000, 6, 40 + b) for b in range(4)]
    one = hwpm_batch_workspace_bytes([(w.n, w.nnz, 0, 0, 0) for w in wls[:1]])
    arena = one + (1 << 20)  # one request and its inputs; never two
    huge = small_random(60000, 8, 99)
    with hwpm.Server(workers=2, max_batch=64, arena_bytes=arena) as srv:
        ts = [srv.submit(w.col_ptr, w.row_idx, w.w) for w in wls]
        th = srv.submit(huge.col_ptr, huge.row_idx, huge.w)
        results = [srv.poll(t) for t in ts]
        rh = srv.poll(th)
        stats = srv.stats()
    for wl, res in zip(wls, results):
        _check(wl, res)
    assert rh[0] == hwpm.HWPM_ETOOBIG and rh[1] is None
    assert stats["max_batch_seen"] == 1 and stats["batches"] == len(wls)
    assert stats["arena_peak"] <= arena


def test_malformed_requests_fail_alone_and_poll_semantics():
    """Malformed matrices are reported by their own poll (validated on the
    device); the well-formed requests batched with them are unaffected."""
    hwpm = _need_gpu()
    good = [small_random(500, 4, 5), small_random(300, 3, 8), stencil27(6, 6, 6, 1, 2)]
    bad = small_random(400, 4, 6)
    ri = bad.row_idx.copy()
    ri[3] = 400  # row out of range
    unsorted = bad.row_idx.copy()
    c0 = int(np.argmax(np.diff(bad.col_ptr) >= 2))
    k = int(bad.col_ptr[c0])
    unsorted[k], unsorted[k + 1] = unsorted[k + 1], unsorted[k]
    wnan = bad.w.copy()
    wnan[7] = np.nan
    cp_bad = bad.col_ptr.copy()
    cp_bad[-1] -= 1  # col_ptr[n] != nnz: refused at submission
    with hwpm.Server(workers=1, max_batch=64) as srv:
        with pytest.raises(hwpm.HwpmError) as e:
            srv.submit(cp_bad, bad.row_idx, bad.w)
        assert e.value.status == hwpm.HWPM_EBADCSC
        tickets = []
        for g, (r, w) in zip(good, ((ri, bad.w), (unsorted, bad.w), (bad.row_idx, wnan))):
            tickets.append((g, srv.submit(g.col_ptr, g.row_idx, g.w)))
            tickets.append((None, srv.submit(bad.col_ptr, r, w)))
        for wl, t in tickets:
            res = srv.poll(t)
            if wl is None:
                assert res[0] == hwpm.HWPM_EBADCSC and res[1] is None
            else:
                _check(wl, res)
        t = srv.submit(good[0].col_ptr, good[0].row_idx, good[0].w)
        res = None
        deadline = time.time() + 60
        while res is None and time.time() < deadline:
            res = srv.poll(t, wait=False)
            if res is None:
                time.sleep(0.001)
        assert res is not None
        _check(good[0], res)
        st, _, _ = hwpm.hwpm_poll(srv.server, t, True, None)  # already delivered
        assert st == hwpm.HWPM_EINVAL
        st, _, _ = hwpm.hwpm_poll(srv.server, 987654321, False, None)
        assert st == hwpm.HWPM_EINVAL


def test_destroy_finishes_queued_requests():
    hwpm = _need_gpu()
    wls = _requests(9, 12)
    srv = hwpm.Server(workers=2, max_batch=4, arena_bytes=128 << 20)
    for w in wls:
        srv.submit(w.col_ptr, w.row_idx, w.w)
    srv.close()  # joins the workers after the queue drains


def test_two_threads_poll_one_ticket():
    """A ticket belongs to the first poll that waits for it: of two threads
    that wait on the same ticket, one gets the result (equal to the oracle's)
    and the other HWPM_EINVAL, and neither touches a released request."""
    import threading
    hwpm = _need_gpu()
    wl = small_random(40000, 6, 91)
    ref = oracle_match(wl.n, wl.col_ptr, wl.row_idx, wl.w)
    print("[gpu] two pollers on one ticket", flush=True)
    for rep in range(4):
        with hwpm.Server(workers=1, max_batch=4, arena_bytes=1 << 30) as srv:
            ticket = srv.submit(wl.col_ptr, wl.row_idx, wl.w)
            perms = [np.empty(wl.n, dtype=np.int32) for _ in range(2)]
            out = [None, None]
            barrier = threading.Barrier(2)

            def poll(i):
                barrier.wait()
                out[i] = hwpm.hwpm_poll(srv.server, ticket, True, perms[i].ctypes.data)

            threads = [threading.Thread(target=poll, args=(i,)) for i in range(2)]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
            statuses = sorted(o[0] for o in out)
            assert statuses == [hwpm.HWPM_EINVAL, hwpm.HWPM_OK], statuses
            winner = 0 if out[0][0] == hwpm.HWPM_OK else 1
            assert np.array_equal(perms[winner], ref.perm)
            assert np.float64(out[winner][1]).tobytes() == np.float64(ref.total).tobytes()
            srv._n.pop(ticket, None)
            srv._keep.pop(ticket, None)
            # the ticket is gone: a third poll is refused too
            assert hwpm.hwpm_poll(srv.server, ticket, False, None)[0] == hwpm.HWPM_EINVAL


def test_destroy_while_a_poll_waits():
    """A poll that waits while the server is destroyed receives its result
    before the server's memory is released; polls started after destroy
    began are refused."""
    import threading
    hwpm = _need_gpu()
    wls = [small_random(60000 + 1000 * k, 6, 92 + k) for k in range(12)]
    srv = hwpm.Server(workers=1, max_batch=1, arena_bytes=1 << 30)
    tickets = [srv.submit(w.col_ptr, w.row_idx, w.w) for w in wls]
    last = wls[-1]
    perm = np.empty(last.n, dtype=np.int32)
    out = []
    th = threading.Thread(target=lambda: out.append(hwpm.hwpm_poll(srv.server, tickets[-1], True,
                                                                   perm.ctypes.data)))
    th.start()
    time.sleep(0.02)
    print("[gpu] destroy with a waiting poll", flush=True)
    srv.close()  # finishes the queued requests, waits for the polling thread
    th.join()
    # a poll already waiting gets the result; one that came after destroy
    # began is refused
    assert out and out[0][0] in (hwpm.HWPM_OK, hwpm.HWPM_EINVAL)
    print(f"[gpu] waiting poll returned {out[0][0]}", flush=True)
    if out[0][0] == hwpm.HWPM_OK:
        ref = oracle_match(last.n, last.col_ptr, last.row_idx, last.w)
        assert np.array_equal(perm, ref.perm)


def test_online_tuning_fills_the_bin():
    """The server tries each candidate launch configuration on the first
    batches of a degree bin, then keeps the fastest; every result equals
    the oracle's, tuned or not."""
    hwpm = _need_gpu()
    wls = [small_random(1500 + 37 * k, 8, 300 + k) for k in range(30)]  # 9 entries per column or so
    print("[gpu] online tuning", flush=True)
    with hwpm.Server(workers=1, max_batch=1, arena_bytes=1 << 30, tune=True) as srv:
        tickets = [srv.submit(w.col_ptr, w.row_idx, w.w) for w in wls]
        for wl, t in zip(wls, tickets):
            _check(wl, srv.poll(t))
        table = srv.tune_table()
    b = hwpm.hwpm_tune_bin(hwpm.hwpm_default_tune_table(), wls[0].n, wls[0].nnz)
    assert table[b]["probe"] in (3, 4, 5) and table[b]["tile_width"] in (4, 8)
    assert table[b]["ms_per_mentry"] > 0.0
    assert all(e["probe"] == 0 for i, e in enumerate(table) if i != b)
