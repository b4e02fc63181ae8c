"""Summarise a rocprofv3 results database (kernel trace, optional counters)
into a short text table for the profiles/ folder.

    python -m paper_1801_09809_amd.profsummary RESULTS.db --command "..." > profiles/X.txt

Reads only the SQLite file rocprofv3 writes (views `kernels`, `pmc_events`).
"""
from __future__ import annotations

import argparse
import sqlite3
import sys
from collections import defaultdict


def kernel_table(con):
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    return [(name, calls, tot, avg, mn, mx, 100.0 * tot / total) for name, calls, tot, avg, mn, mx in rows]


def counter_table(con):
    try:
        rows = con.execute(
            "select k.name, p.counter_name, avg(p.value), count(*) from pmc_events p "
            "join kernels k on p.event_id = k.event_id group by k.name, p.counter_name").fetchall()
    except sqlite3.Error:
        return []
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--command", default="", help="the command that produced the database")
    ap.add_argument("--top", type=int, default=20)
    args = ap.parse_args(argv)
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
        by = defaultdict(dict)
        for name, cname, val, cnt in ct:
            by[name][cname] = (val, cnt)
        for name, d in by.items():
            vals = ", ".join(f"{c}={v:.6g} (n={n})" for c, (v, n) in sorted(d.items()))
            print(f"  {name[:90]}: {vals}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
