"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/hwpm.h declares, and its host-side argument logic answers
without touching a device."""
import ctypes
import os
import re
import subprocess

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
    found = re.findall(r"#define (HWPM_E[A-Z]+|HWPM_OK|HWPM_PENDING)\s+(-?\d+)", text)
    assert len(found) == 10
    for name, val in found:
        assert getattr(hwpm, name) == int(val), name
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 1):
        assert hwpm.hwpm_strerror(code) not in ("", "unknown status")
    assert hwpm.hwpm_strerror(12345) == "unknown status"


def test_struct_layouts():
    # the ctypes mirrors must match the C layout (offsets of the last fields)
    assert ctypes.sizeof(hwpm.hwpm_csc) == 40
    assert ctypes.sizeof(hwpm.hwpm_options) == 32
    s = hwpm.hwpm_stats
    assert s.init_weight.offset == 40 and s.ms_check.offset == 56
    assert s.round_candidates.offset == 112
    assert ctypes.sizeof(s) == 112 + 4 * 4 * hwpm.MAX_ROUND_STATS


_STRUCTS = ("hwpm_csc", "hwpm_options", "hwpm_stats", "hwpm_item_stats", "hwpm_server_options",
            "hwpm_request_info", "hwpm_server_stats", "hwpm_tune_table")


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what gcc
    lays out from include/hwpm.h."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hwpm.h"', "int main(void) {"]
    for sname in _STRUCTS:
        cls = getattr(hwpm, sname)
        lines.append(f'printf("{sname} sizeof %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        sname, fname, val = line.split()
        cls = getattr(hwpm, sname)
        got = ctypes.sizeof(cls) if fname == "sizeof" else getattr(cls, fname).offset
        assert got == int(val), (sname, fname, got, val)
        seen += 1
    assert seen == sum(len(getattr(hwpm, s)._fields_) + 1 for s in _STRUCTS)


def test_server_host_argument_checks():
    lib = hwpm.load_library()
    assert lib.hwpm_server_create(None, None) == hwpm.HWPM_EINVAL
    o = hwpm.hwpm_server_default_options()
    assert (o.workers, o.max_batch, o.arena_bytes, o.solve.check_csc) == (2, 64, 8 << 30, 1)
    s = ctypes.c_void_p()
    for field, bad in (("workers", 0), ("workers", 17), ("max_batch", 0), ("arena_bytes", 1000)):
        ob = hwpm.hwpm_server_default_options()
        setattr(ob, field, bad)
        assert lib.hwpm_server_create(ctypes.byref(s), ctypes.byref(ob)) == hwpm.HWPM_EINVAL
    st, _ = hwpm.hwpm_submit(0, 3, 3, 1, 1, 1)
    assert st == hwpm.HWPM_EINVAL
    st, _, _ = hwpm.hwpm_poll(0, 1, False, None)
    assert st == hwpm.HWPM_EINVAL
    assert hwpm.hwpm_server_destroy(0) == hwpm.HWPM_OK
    assert lib.hwpm_server_get_stats(None, None) == hwpm.HWPM_EINVAL


@pytest.mark.skipif(torch.cuda.is_available(), reason="needs a machine without a GPU")
def test_server_without_device_fails_cleanly():
    with pytest.raises(hwpm.HwpmError) as e:
        hwpm.hwpm_server_create(None)
    assert e.value.status == hwpm.HWPM_EDEVICE


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
    assert lib.hwpm_autotune(None, None, None, None, None, None, None, 0) == hwpm.HWPM_EINVAL
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


def test_tune_table_bins():
    """Degree bins of the tuning table (host code only): bounds 4, 8, 16, 32,
    64 entries per column and one open bin; every entry starts untuned."""
    t = hwpm.hwpm_default_tune_table()
    assert [float(x) for x in t.max_degree[:5]] == [4.0, 8.0, 16.0, 32.0, 64.0]
    assert all(p == 0 for p in t.probe) and all(x == 0 for x in t.tile_width)
    cases = [(0, 0, 0), (100, 0, 0), (100, 400, 0), (100, 401, 1), (100, 800, 1), (100, 1600, 2),
             (1 << 20, 17825657, 3), (1_000_000, 26_463_592, 3), (10, 641, 5), (10, 640, 4)]
    for n, nnz, b in cases:
        assert hwpm.hwpm_tune_bin(t, n, nnz) == b, (n, nnz)
