"""Benchmark: 4-cycle-search edges/s of the HWPM weight-improvement rounds on one GPU.

A step is one whole hwpm_improve call on the resident synthetic matrix: set-up
(mates, matched weights, long-column table), every round of cycle search +
per-root argmax (Steps A-C), conflict resolution (Step D) and flips, until a
round flips nothing, then the fixed-order total and the output copy.  The
inputs (CSC and the starting perfect matching) are in HBM before the timed
region; the CSC is validated once, before it.

value = nnz * rounds / (wall time per step)  [edges scanned per second]

The JSON line also carries the roofline of the dominant kernel (the cycle
search) from HIP events recorded by the library on its stream, and a CPU
baseline: the oracle on the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak


def search_bytes(nnz: int, n: int) -> float:
    """Algorithmic bytes of one full cycle-search launch with the transposed
    probe: each edge is visited twice per round (in its column for the pruned
    half: row index 4 B + mate column 4 B; in the row list of m_j: 4 B), i.e.
    8 B per entry, plus 16 B per column (column pointer, m_j, w(m_j, j)).  The
    24 B per closing-edge hit are left out (a lower bound: hits are rare on
    the random workload)."""
    return 8.0 * nnz + 16.0 * n


def load_traffic(kernel: str):
    """HBM bytes per launch measured by rocprofv3 counters, if recorded for the
    current kernel source (profiles/traffic.json holds the source hash)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        import hashlib
        with open(path) as f:
            rec = json.load(f).get(kernel)
        src = os.path.join(ROOT, "paper_1801_09809_amd", "csrc", "hwpm_kernels.hip")
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if rec and rec.get("kernel_src_sha") == sha:
            return float(rec["bytes_per_launch"])
    except Exception:
        return None
    return None


def cpu_baseline(wl) -> dict:
    """The oracle (single thread) on the same workload from the same matching."""
    from oracle import oracle_improve
    t0 = time.perf_counter()
    ref = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted)
    dt = time.perf_counter() - t0
    return {"value": wl.nnz * ref.rounds / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of {wl.name} ({ref.rounds} rounds, {dt:.2f} s)",
            "rounds": ref.rounds}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=1)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--probe", type=int, default=0,
                    help="0 default, 1 column search, 2 row lists, 3 chunked row lists")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the per-stage HIP events (roofline fields become null)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB three times "
                         "(a device copy kernel of known size, to scale rocprofv3 byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md but not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1801_09809_amd import hwpm
    from workloads import workload

    wl = workload(args.workload)
    print(f"[bench] workload {args.workload}: {wl.name} n={wl.n} nnz={wl.nnz}", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    cp = torch.from_numpy(wl.col_ptr).to(dev)
    ri = torch.from_numpy(wl.row_idx).to(dev)
    w = torch.from_numpy(wl.w).to(dev)
    mate = torch.from_numpy(wl.planted).to(dev)
    perm = torch.empty_like(mate)
    solver = hwpm.Solver(0)
    st = solver.check_csc(cp, ri, w)
    if st != hwpm.HWPM_OK:
        raise hwpm.HwpmError(st, "hwpm_check_csc")

    def step(full=True, timing=not args.no_timing):
        # full rounds: every column searched every round (search throughput)
        return solver.improve(cp, ri, w, mate, perm_out=perm, check_csc=False, timing=timing,
                              tile_width=args.tile, probe=args.probe, full_search=full)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step().stats)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    rounds = stats[0]["rounds"]
    assert all(s["rounds"] == rounds for s in stats)
    edges = float(wl.nnz) * rounds
    print(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step, rounds={rounds}", file=sys.stderr, flush=True)

    out = {
        "metric": "4-cycle-search edges/s (1 GPU)",
        "value": edges / (ms_step / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "nnz": wl.nnz, "rounds": rounds,
                   "cycles_applied": stats[0]["cycles_applied"],
                   "start": "planted perfect matching (permuted diagonal)",
                   "tile_width": args.tile or 4, "probe": args.probe or 3},
    }
    if not args.no_timing:
        ms_search = float(np.mean([s["ms_search"] for s in stats]))
        launch_ms = ms_search / rounds
        alg = search_bytes(wl.nnz, wl.n)
        achieved = alg / (launch_ms / 1e3) / 1e9
        traffic = load_traffic("k_search_short")
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": "k_search_chunk (Steps A-C)",
                           "algorithmic_bytes_per_launch": alg, "avg_launch_ms": launch_ms}
        out["search_edges_per_s"] = edges / (ms_search / 1e3)
        out["ms_breakdown"] = {k: float(np.mean([s[k] for s in stats])) for k in
                               ("ms_setup", "ms_transpose", "ms_search", "ms_resolve", "ms_apply",
                                "ms_final", "ms_total")}
    # the library's default solve (incremental rounds: identical result)
    if (args.probe or 3) == 3:
        inc = [step(full=False, timing=False) for _ in range(max(2, args.warmup))]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps = max(3, args.steps // 2)
        for _ in range(reps):
            inc_stats = step(full=False, timing=False).stats
        torch.cuda.synchronize()
        out["solve_ms_incremental"] = 1e3 * (time.perf_counter() - t1) / reps
        out["incremental_roots_searched"] = int(sum(inc_stats["round_roots"]))
        assert inc_stats["round_applied"] == stats[0]["round_applied"]
    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    solver.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
