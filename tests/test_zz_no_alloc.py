"""GPU test of hwpm_improve_static, the allocation-free form of hwpm_improve
(its workspace is the library's fixed device array): called through the C
ABI, its outputs equal hwpm_improve's bit for bit on two calls in a row, the
second with a smaller matrix, and a matrix whose workspace exceeds the array
is refused with its output untouched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import small_random, stencil27  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _both(solver, wl, probe):
    from paper_1801_09809_amd import hwpm
    dev = solver.device
    cp, ri, w, mate = _dev(wl.col_ptr, dev), _dev(wl.row_idx, dev), _dev(wl.w, dev), _dev(wl.planted, dev)
    print(f"[gpu] static workspace {wl.name} n={wl.n} nnz={wl.nnz} probe={probe}", flush=True)
    ref = solver.improve(cp, ri, w, mate, probe=probe)
    out = torch.full((wl.n,), -7, dtype=torch.int32, device=dev)
    opt = hwpm.Solver.options(probe=probe)
    st, total, stats = hwpm.hwpm_improve_static(solver.handle, wl.n, wl.nnz, cp.data_ptr(), ri.data_ptr(),
                                                w.data_ptr(), mate.data_ptr(), out.data_ptr(), opt)
    torch.cuda.synchronize()
    assert st == hwpm.HWPM_OK
    assert torch.equal(out, ref.perm)
    assert np.float64(total).tobytes() == np.float64(ref.total).tobytes()
    got = stats.as_dict()
    for k in ("rounds", "cycles_applied", "round_candidates", "round_applied", "init_weight"):
        assert got[k] == ref.stats[k], k


@pytest.mark.parametrize("probe", [1, 3, 5])
def test_static_workspace_equals_caller_workspace(probe):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1801_09809_amd import hwpm
    solver = hwpm.Solver(0)
    try:
        big = stencil27(40, 40, 30, 2201, 3201, name="stencil_40x40x30")      # 48,000 columns
        small = small_random(9001, 7, 2202)
        for wl in (big, small):  # the second call is smaller: the array keeps the first call's contents
            _both(solver, wl, probe)
        # beyond the array: refused, output untouched
        n, nnz = 1_000_000, 4_000_000
        need = hwpm.hwpm_workspace_bytes(n, nnz)
        assert need > hwpm.STATIC_SCRATCH_BYTES
        dev = solver.device
        cp = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        cp[-1] = nnz
        ri = torch.zeros(nnz, dtype=torch.int32, device=dev)
        w = torch.zeros(nnz, dtype=torch.float64, device=dev)
        mate = torch.arange(n, dtype=torch.int32, device=dev)
        out = torch.full((n,), -7, dtype=torch.int32, device=dev)
        st, _, _ = hwpm.hwpm_improve_static(solver.handle, n, nnz, cp.data_ptr(), ri.data_ptr(), w.data_ptr(),
                                            mate.data_ptr(), out.data_ptr())
        assert st == hwpm.HWPM_ETOOBIG
        assert bool((out == -7).all())
    finally:
        solver.close()
