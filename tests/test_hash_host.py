"""Host build of the kernels' LDS hash sets (paper_1801_09809_amd/csrc/hwpm_hash.h).

The header is compiled with g++ for the host and driven by
tests/host/hash_host_test.cpp: every insert and lookup loop must end on full,
near-full and duplicate-key tables, and lookups must return exactly what was
inserted.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_hash_sets_on_host(tmp_path):
    exe = tmp_path / "hash_host_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1801_09809_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "hash_host_test.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"
