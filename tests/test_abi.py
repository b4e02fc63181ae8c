"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/hwpm.h declares, and its host-side argument logic answers
without touching a device."""
import ctypes
import os
import re

import pytest
import torch

from paper_1801_09809_amd import hwpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hwpm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hwpm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = hwpm.load_library()
    declared = _declared()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in hwpm.h but not exported"
    assert sorted(hwpm.EXPORTED) == declared


def test_status_codes_match_header():
    text = open(HEADER).read()
    for name, val in re.findall(r"#define (HWPM_E[A-Z]+|HWPM_OK)\s+(-?\d+)", text):
        assert getattr(hwpm, name) == int(val), name
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert hwpm.hwpm_strerror(code) not in ("", "unknown status")
    assert hwpm.hwpm_strerror(12345) == "unknown status"


def test_struct_layouts():
    # the ctypes mirrors must match the C layout (offsets of the last fields)
    assert ctypes.sizeof(hwpm.hwpm_csc) == 40
    assert ctypes.sizeof(hwpm.hwpm_options) == 28
    s = hwpm.hwpm_stats
    assert s.init_weight.offset == 40 and s.ms_check.offset == 56
    assert s.round_candidates.offset == 104
    assert ctypes.sizeof(s) == 104 + 4 * 4 * hwpm.MAX_ROUND_STATS


def test_default_options():
    o = hwpm.hwpm_default_options()
    assert (o.max_rounds, o.check_csc, o.timing, o.tile_width, o.probe, o.mcm_plain,
            o.full_search) == (0, 1, 0, 0, 0, 0, 0)


def test_workspace_bytes():
    b0 = hwpm.hwpm_workspace_bytes(0, 0)
    b1 = hwpm.hwpm_workspace_bytes(1000, 9000)
    b2 = hwpm.hwpm_workspace_bytes(1 << 20, 17_825_657)
    assert 0 < b0 < b1 < b2
    # O(nnz + n): row lists, their staging and per-entry mates; per-vertex state
    assert b2 < 60 * 17_825_657 + 400 * (1 << 20)
    with pytest.raises(hwpm.HwpmError) as e:
        hwpm.hwpm_workspace_bytes(-1, 0)
    assert e.value.status == hwpm.HWPM_EINVAL
    with pytest.raises(hwpm.HwpmError) as e:
        hwpm.hwpm_workspace_bytes(10, 1 << 41)
    assert e.value.status == hwpm.HWPM_ETOOBIG


def test_host_argument_checks():
    # no handle, no csc: rejected on the host before any device call
    st, _, _ = hwpm.hwpm_improve(0, 3, 3, 1, 1, 1, 1, 1, 1, 1 << 20)
    assert st == hwpm.HWPM_EINVAL
    lib = hwpm.load_library()
    assert lib.hwpm_improve(ctypes.c_void_p(1), None, None, None, None, None, None, None, 0) == hwpm.HWPM_EINVAL
    assert hwpm.hwpm_check_csc(0, 3, 3, 1, 1, 1, 1, 1 << 20) == hwpm.HWPM_EINVAL
    assert lib.hwpm_create(None, 0, None) == hwpm.HWPM_EINVAL
    assert hwpm.hwpm_destroy(0) == hwpm.HWPM_OK


@pytest.mark.skipif(torch.cuda.is_available(), reason="needs a machine without a GPU")
def test_create_without_device_fails_cleanly():
    with pytest.raises(hwpm.HwpmError) as e:
        hwpm.hwpm_create(0, None)
    assert e.value.status == hwpm.HWPM_EDEVICE


def test_solver_refuses_without_gpu():
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        hwpm.Solver(0)
