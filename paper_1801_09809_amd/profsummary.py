"""Summarise rocprofv3 results databases into short text for the profiles/
folder, and derive the HBM traffic of a kernel from two counter passes.

    python -m paper_1801_09809_amd.profsummary trace RESULTS.db --command "..."
    python -m paper_1801_09809_amd.profsummary pmc --fetch FETCH.db --write WRITE.db --copy-bytes N
    python -m paper_1801_09809_amd.profsummary issue SQ.db --kernel k_search_filter --cus 256 --xcds 8
    python -m paper_1801_09809_amd.profsummary traffic --fetch FETCH.db --write WRITE.db \
        --kernel "k_search_filter<4, 8, true, false>" --kernel k_search_medium --name search_stage --copy-bytes N \
        --source csrc/hwpm_search.hip,csrc/hwpm_device.h,csrc/hwpm_hash.h,csrc/hwpm_internal.h \
        --workload random_n1048576_d16 --probe 5 --out profiles/traffic.json

Reads only the SQLite files rocprofv3 writes (views `kernels` and
`counters_collection`).  Counter values are summed over the rows of one
dispatch, then averaged over the dispatches of a kernel.

Traffic calibration: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled
by what the same counters read for the runtime's device-to-device copy kernel
of a known size in the same run (algorithmic bytes / counted bytes), so the
figure is in true HBM bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import sqlite3
import sys
from collections import defaultdict

COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_table(con):
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    return [(name, calls, tot, avg, mn, mx, 100.0 * tot / total) for name, calls, tot, avg, mn, mx in rows]


def counter_table(con):
    """{kernel name: {counter: (average per dispatch, dispatches)}}; per dispatch,
    values of the same counter are summed."""
    try:
        rows = con.execute(
            "select kernel_name, counter_name, dispatch_id, sum(value) from counters_collection "
            "group by kernel_name, counter_name, dispatch_id").fetchall()
    except sqlite3.Error:
        return {}
    acc = defaultdict(lambda: defaultdict(list))
    for name, cname, _disp, val in rows:
        acc[name][cname].append(val)
    return {name: {c: (sum(v) / len(v), len(v)) for c, v in d.items()} for name, d in acc.items()}


def dispatch_values(con, counter):
    """[(kernel name, value)] per dispatch, in dispatch order."""
    rows = con.execute(
        "select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name = ? "
        "group by dispatch_id order by dispatch_id", (counter,)).fetchall()
    return [(name, val) for name, _d, val in rows]


def match_kernel(names, key):
    hits = sorted({n for n in names if key in n})
    if len(hits) != 1:
        raise SystemExit(f"kernel key {key!r} matches {hits}")
    return hits[0]


def cmd_trace(args) -> int:
    con = sqlite3.connect(args.db)
    if args.command:
        print(f"command: {args.command}")
    print("kernel trace (durations in microseconds)")
    print(f"{'calls':>6} {'total_us':>12} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}  kernel")
    for name, calls, tot, avg, mn, mx, pct in kernel_table(con)[: args.top]:
        print(f"{calls:6d} {tot / 1e3:12.1f} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} "
              f"{pct:6.1f}  {name[:110]}")
    ct = counter_table(con)
    if ct:
        print("\ncounters (average per dispatch)")
        for name, d in ct.items():
            vals = ", ".join(f"{c}={v:.6g} (n={n})" for c, (v, n) in sorted(d.items()))
            print(f"  {name[:90]}: {vals}")
    return 0


def _calibrated(db, counter, kernel_key, copy_bytes):
    con = sqlite3.connect(db)
    vals = dispatch_values(con, counter)
    if not vals:
        raise SystemExit(f"{db}: no {counter} values")
    kname = match_kernel({n for n, _ in vals}, kernel_key)
    kv = [v for n, v in vals if n == kname]
    # the calibration copies are the largest copy-kernel dispatches
    cv = sorted((v for n, v in vals if n.startswith(COPY_KERNEL)), reverse=True)[:3]
    if not cv:
        raise SystemExit(f"{db}: no {COPY_KERNEL} dispatch to calibrate with")
    copy_kib = sum(cv) / len(cv)
    factor = (copy_bytes / 1024.0) / copy_kib
    per_launch_kib = sum(kv) / len(kv)
    return kname, per_launch_kib, copy_kib, factor, len(kv)


def cmd_traffic(args) -> int:
    """Traffic of one stage: the kernels named by --kernel (one substring
    each), each launched once per stage; their per-dispatch averages add."""
    keys = list(args.kernel)
    h = hashlib.sha256()
    for f in args.source.split(","):
        h.update(open(f, "rb").read())
    sha = h.hexdigest()[:16]
    kernels = {}
    read_b = write_b = 0.0
    f_copy = w_copy = f_fac = w_fac = None
    for key in keys:
        kname, f_kib, f_copy, f_fac, nf = _calibrated(args.fetch, "FETCH_SIZE", key, args.copy_bytes)
        _, w_kib, w_copy, w_fac, nw = _calibrated(args.write, "WRITE_SIZE", key, args.copy_bytes)
        kernels[kname] = {"fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
                          "dispatches": [nf, nw]}
        read_b += f_kib * 1024.0 * f_fac
        write_b += w_kib * 1024.0 * w_fac
    rec = {"kernels": kernels, "kernel_src_sha": sha, "bytes_per_launch": read_b + write_b,
           "read_bytes_per_launch": read_b, "write_bytes_per_launch": write_b,
           "copy_bytes": args.copy_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
           "fetch_factor": f_fac, "write_factor": w_fac, "workload": args.workload, "probe": args.probe, "command": args.command}
    data = {}
    try:
        with open(args.out) as f:
            data = json.load(f)
    except (OSError, ValueError):
        pass
    data[args.name] = rec
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(rec, indent=1))
    return 0


def _copy_factor(vals, copy_bytes):
    cv = sorted((v for n, v in vals if n.startswith(COPY_KERNEL)), reverse=True)[:3]
    if not cv:
        raise SystemExit(f"no {COPY_KERNEL} dispatch to calibrate with")
    copy_kib = sum(cv) / len(cv)
    return copy_kib, (copy_bytes / 1024.0) / copy_kib


def cmd_pmc(args) -> int:
    """Per-kernel HBM traffic of every kernel in two counter passes, raw and
    calibrated, averaged over each kernel's dispatches (MB = 10^6 bytes)."""
    fv = dispatch_values(sqlite3.connect(args.fetch), "FETCH_SIZE")
    wv = dispatch_values(sqlite3.connect(args.write), "WRITE_SIZE")
    f_copy, f_fac = _copy_factor(fv, args.copy_bytes)
    w_copy, w_fac = _copy_factor(wv, args.copy_bytes)
    fk, wk = defaultdict(list), defaultdict(list)
    for n, v in fv:
        fk[n].append(v)
    for n, v in wv:
        wk[n].append(v)
    if args.command_fetch:
        print(f"command (FETCH_SIZE pass): {args.command_fetch}")
    if args.command_write:
        print(f"command (WRITE_SIZE pass): {args.command_write}")
    mib = args.copy_bytes / 1048576
    print(f"calibration: three device copies of {mib:.0f} MiB read FETCH_SIZE {f_copy:.0f} KiB and "
          f"WRITE_SIZE {w_copy:.0f} KiB each,")
    print(f"so counted KiB are scaled by {f_fac:.4f} (reads) and {w_fac:.4f} (writes); values below are "
          "per dispatch, averaged over dispatches.")
    print("note: a kernel's WRITE_SIZE also counts lines the previous kernel left dirty in the caches, "
          "so writes are attributed loosely.\n")
    print(f"{'fetch_MB':>10} {'write_MB':>10} {'calib_read_MB':>14} {'calib_write_MB':>15} {'n':>4}  kernel")
    rows = []
    for n in set(fk) | set(wk):
        f = sum(fk[n]) / len(fk[n]) if fk[n] else 0.0
        w = sum(wk[n]) / len(wk[n]) if wk[n] else 0.0
        rows.append((f * f_fac + w * w_fac, n, f, w, max(len(fk[n]), len(wk[n]))))
    for _, n, f, w, cnt in sorted(rows, reverse=True)[: args.top]:
        print(f"{f * 1.024e-3:10.2f} {w * 1.024e-3:10.2f} {f * f_fac * 1.024e-3:14.2f} "
              f"{w * w_fac * 1.024e-3:15.2f} {cnt:4d}  {n[:100]}")
    return 0


def cmd_issue(args) -> int:
    """Instruction mix of one kernel from an SQ counter pass, per wave and
    per compute unit.  A wave64 vector instruction occupies its 16-lane SIMD
    for 4 cycles, so a CU (4 SIMDs) issues at most one per cycle: the vector
    instructions per CU over the kernel's cycles is the vector unit's busy
    fraction.  GRBM_GUI_ACTIVE is summed over the XCDs."""
    con = sqlite3.connect(args.db)
    ct = counter_table(con)
    name = match_kernel(ct.keys(), args.kernel)
    d = {c: v for c, (v, _n) in ct[name].items()}
    n = min(nn for _v, nn in ct[name].values())
    if args.command:
        print(f"command: {args.command}")
    print(f"kernel: {name}")
    print(f"dispatches: {n}; counters averaged per dispatch (summed over the chip)")
    for c in sorted(d):
        print(f"  {c:24s} {d[c]:14.6g}")
    waves = d.get("SQ_WAVES", 0.0)
    if waves:
        for c, label in (("SQ_INSTS_VALU", "vector"), ("SQ_INSTS_SALU", "scalar"),
                         ("SQ_INSTS_VMEM_RD", "vector memory reads")):
            if c in d:
                print(f"{label} instructions per wave: {d[c] / waves:.1f}")
    if "GRBM_GUI_ACTIVE" in d and "SQ_INSTS_VALU" in d:
        cycles = d["GRBM_GUI_ACTIVE"] / args.xcds
        per_cu = d["SQ_INSTS_VALU"] / args.cus
        print(f"kernel cycles (per XCD): {cycles:.0f}; vector instructions per CU: {per_cu:.0f}; "
              f"vector issue busy: {per_cu / cycles:.2f}")
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", default="", help="the command that produced the database")
    t.add_argument("--top", type=int, default=25)
    r = sub.add_parser("traffic")
    r.add_argument("--fetch", required=True, help="database of the FETCH_SIZE pass")
    r.add_argument("--write", required=True, help="database of the WRITE_SIZE pass")
    r.add_argument("--kernel", action="append", required=True,
                   help="a substring naming one kernel of the stage (once per kernel)")
    r.add_argument("--name", required=True, help="key of the record in the output file")
    r.add_argument("--copy-bytes", type=int, required=True, help="bytes of each calibration copy")
    r.add_argument("--source", required=True,
                   help="comma-separated source files of the kernels (their joint hash is recorded)")
    r.add_argument("--out", required=True)
    r.add_argument("--workload", required=True, help="name of the workload the passes ran on")
    r.add_argument("--probe", type=int, required=True, help="the probe the passes ran with")
    r.add_argument("--command", default="")
    m = sub.add_parser("pmc")
    m.add_argument("--fetch", required=True, help="database of the FETCH_SIZE pass")
    m.add_argument("--write", required=True, help="database of the WRITE_SIZE pass")
    m.add_argument("--copy-bytes", type=int, required=True, help="bytes of each calibration copy")
    m.add_argument("--command-fetch", default="")
    m.add_argument("--command-write", default="")
    m.add_argument("--top", type=int, default=25)
    q = sub.add_parser("issue")
    q.add_argument("db", help="database of an SQ counter pass")
    q.add_argument("--kernel", required=True, help="substring naming one kernel")
    q.add_argument("--cus", type=int, default=256)
    q.add_argument("--xcds", type=int, default=8)
    q.add_argument("--command", default="")
    args = ap.parse_args(argv)
    return {"trace": cmd_trace, "traffic": cmd_traffic, "pmc": cmd_pmc, "issue": cmd_issue}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
