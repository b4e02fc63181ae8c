"""CPU tests of the profile summariser (paper_1801_09809_amd/profsummary.py) on
small synthetic databases with the two tables it reads from rocprofv3 output:
kernel durations and per-dispatch counter values."""
import json
import sqlite3

import pytest

from paper_1801_09809_amd import profsummary as ps

COPY = ps.COPY_KERNEL + "(void*, void const*)"


def _db(path, kernels, counters):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)", kernels)
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "dispatch_id integer, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", counters)
    con.commit()
    con.close()
    return str(path)


@pytest.fixture()
def passes(tmp_path):
    """FETCH_SIZE / WRITE_SIZE passes: a search kernel launched twice, a
    second kernel once, and three calibration copies of 1 MiB that count
    512 KiB fetched (factor 2) and 1024 KiB written (factor 1).  Counter
    rows of one dispatch are split in two, as rocprofv3 reports per-block
    instances."""
    mib = 1024.0

    def rows(counter, search_kib, other_kib, copy_kib):
        out, d = [], 0
        for kib in search_kib:
            d += 1
            out += [("k_search_chunk<4, 8>", counter, d, kib / 2), ("k_search_chunk<4, 8>", counter, d, kib / 2)]
        d += 1
        out.append(("k_tp_hist", counter, d, other_kib))
        for _ in range(3):
            d += 1
            out.append((COPY, counter, d, copy_kib))
        d += 1
        out.append((COPY, counter, d, 1.0))  # a small copy: not a calibration copy
        return out

    kern = [("k_search_chunk<4, 8>", 3000), ("k_search_chunk<4, 8>", 5000), ("k_tp_hist", 1000)]
    fetch = _db(tmp_path / "f.db", kern, rows("FETCH_SIZE", [100.0, 300.0], 50.0, mib / 2))
    write = _db(tmp_path / "w.db", kern, rows("WRITE_SIZE", [10.0, 30.0], 5.0, mib))
    return fetch, write


def test_trace_table(passes, capsys):
    fetch, _ = passes
    assert ps.main(["trace", fetch, "--command", "cmd"]) == 0
    out = capsys.readouterr().out
    assert out.startswith("command: cmd")
    line = [x for x in out.splitlines() if "k_search_chunk" in x][0].split()
    # 2 calls, 8 us total, 4 us average, 3 and 5 us extremes, 8/9 of the time
    assert line[:6] == ["2", "8.0", "4.00", "3.00", "5.00", "88.9"]


def test_traffic_record_is_calibrated(passes, tmp_path):
    fetch, write = passes
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    out = tmp_path / "traffic.json"
    assert ps.main(["traffic", "--fetch", fetch, "--write", write, "--kernel", "k_search_chunk",
                    "--name", "search_stage", "--copy-bytes", str(1 << 20), "--source", str(src),
                    "--out", str(out), "--workload", "wl", "--probe", "5"]) == 0
    rec = json.loads(out.read_text())["search_stage"]
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    # mean of 100 and 300 KiB fetched, x2; mean of 10 and 30 KiB written, x1
    assert rec["read_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)
    assert rec["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2 + 20.0 * 1024)
    assert rec["workload"] == "wl" and rec["probe"] == 5 and len(rec["kernel_src_sha"]) == 16


def test_traffic_rejects_ambiguous_kernel_key(passes, tmp_path):
    fetch, write = passes
    src = tmp_path / "k.hip"
    src.write_text("x")
    with pytest.raises(SystemExit):
        ps.main(["traffic", "--fetch", fetch, "--write", write, "--kernel", "k_",
                 "--name", "s", "--copy-bytes", str(1 << 20), "--source", str(src),
                 "--out", str(tmp_path / "t.json"), "--workload", "wl", "--probe", "5"])


def test_pmc_table(passes, capsys):
    fetch, write = passes
    assert ps.main(["pmc", "--fetch", fetch, "--write", write, "--copy-bytes", str(1 << 20)]) == 0
    out = capsys.readouterr().out
    assert "scaled by 2.0000 (reads) and 1.0000 (writes)" in out
    line = [x for x in out.splitlines() if "k_search_chunk" in x][0].split()
    # raw 200 KiB fetched and 20 KiB written per dispatch; calibrated 400 and 20 KiB
    assert [float(v) for v in line[:4]] == pytest.approx([0.2048, 0.02048, 0.4096, 0.02048], abs=6e-3)
    assert line[4] == "2"


def test_traffic_of_a_two_kernel_stage(passes, tmp_path):
    """--kernel once per kernel of the stage (a key may hold commas, as
    template arguments do); the per-dispatch averages add."""
    fetch, write = passes
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    out = tmp_path / "traffic.json"
    assert ps.main(["traffic", "--fetch", fetch, "--write", write, "--kernel", "k_search_chunk<4, 8>",
                    "--kernel", "k_tp_hist", "--name", "stage", "--copy-bytes", str(1 << 20),
                    "--source", str(src), "--out", str(out), "--workload", "wl", "--probe", "5"]) == 0
    rec = json.loads(out.read_text())["stage"]
    # (200 + 50) KiB fetched x2, (20 + 5) KiB written x1
    assert rec["read_bytes_per_launch"] == pytest.approx(250.0 * 1024 * 2)
    assert rec["write_bytes_per_launch"] == pytest.approx(25.0 * 1024)
    assert len(rec["kernels"]) == 2


def test_issue_summary(tmp_path, capsys):
    """Instruction mix per wave and the vector unit's busy fraction: 100
    waves of 300 vector instructions on 4 CUs is 7,500 per CU; over 10,000
    cycles per die (GRBM summed over 2 dies) that is 0.75."""
    counters = []
    for d in (1, 2):  # two dispatches, each counter split over two rows
        for c, v in (("SQ_WAVES", 100.0), ("SQ_INSTS_VALU", 30000.0), ("SQ_INSTS_SALU", 5000.0),
                     ("GRBM_GUI_ACTIVE", 20000.0)):
            counters += [("k_search_filter<4, 8, true, false>", c, d, v / 2)] * 2
    db = _db(tmp_path / "sq.db", [("k_search_filter<4, 8, true, false>", 1000)], counters)
    assert ps.main(["issue", db, "--kernel", "k_search_filter", "--cus", "4", "--xcds", "2"]) == 0
    out = capsys.readouterr().out
    assert "vector instructions per wave: 300.0" in out
    assert "scalar instructions per wave: 50.0" in out
    assert "vector issue busy: 0.75" in out
