"""Write tests/golden/rmat_scale22_converged.json from the oracle alone.

The R-MAT scale-22 workload (edge factor 16, about 69.4 M entries) needs 119
rounds from its planted matching; the sequential oracle takes minutes for
that, too long for a test, so its result is stored once.  This script calls
only the seeded input generators and the oracle (never the HIP library):

    python tests/golden/make_rmat_golden.py

The record holds digests of the generated input (so a test can tell that it
regenerated the same matrix), and of the oracle's result: the permutation's
sha256, the bit patterns of the initial and final totals, the round count,
the cycles flipped and the per-round candidate and flip counts (Section 5.3,
Algorithm 2: rounds until one flips nothing), for the uncapped loop and for
the paper's cap of 10 rounds (Section 4).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "rmat_scale22_converged.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def bits(x: float) -> str:
    return np.float64(x).tobytes()[::-1].hex()  # big-endian hex of the binary64 pattern


def record(res) -> dict:
    return {"perm_sha256": digest(res.perm.astype(np.int32)), "total_bits": bits(res.total),
            "total": float(res.total), "init_weight_bits": bits(res.init_weight),
            "rounds": int(res.rounds), "hit_round_cap": bool(res.hit_round_cap),
            "cycles_applied": int(res.cycles_applied),
            "round_candidates": [int(x) for x in res.round_candidates],
            "round_applied": [int(x) for x in res.round_applied]}


def main() -> int:
    from oracle import oracle_improve
    from workloads import workload

    t0 = time.perf_counter()
    wl = workload(3)
    print(f"generated {wl.name}: n={wl.n} nnz={wl.nnz} ({time.perf_counter() - t0:.1f} s)", flush=True)
    out = {"about": "Oracle result (never the GPU's) for the R-MAT scale-22 workload from its planted "
                    "matching; written by tests/golden/make_rmat_golden.py.  Bit patterns are big-endian "
                    "hex of binary64 values.",
           "workload": wl.name, "n": wl.n, "nnz": wl.nnz,
           "input_sha256": {"col_ptr": digest(wl.col_ptr), "row_idx": digest(wl.row_idx),
                            "w": digest(wl.w), "planted": digest(wl.planted)}}
    for cap, key in ((0, "converged"), (10, "maxiters_10")):
        t0 = time.perf_counter()
        res = oracle_improve(wl.n, wl.col_ptr, wl.row_idx, wl.w, wl.planted, cap)
        print(f"oracle max_rounds={cap}: {res.rounds} rounds, {res.cycles_applied} flips "
              f"({time.perf_counter() - t0:.1f} s)", flush=True)
        out[key] = record(res)
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    os.replace(tmp, OUT)
    print(f"wrote {OUT}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
