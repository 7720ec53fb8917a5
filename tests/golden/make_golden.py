"""Write tests/golden/oracle_values.json: exact per(A) of the seeded full-size workloads.

Calls only the oracle (C Algorithm H_per, cross-checked against the frontier DP where that
is fast) on inputs from the seeded generators. Run: python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import native, per_dp  # noqa: E402


def main():
    threads = os.cpu_count() or 8
    out = {"_comment": "exact per(A) from the oracle (C Algorithm H_per); keys name the seeded workload"}
    groups = {
        "n24": [(f"cubic24_seed{s}", A) for s, A in zip(range(10), W.config_n24())],
        "n60": W.config_n60(16),
        "n80": W.config_n80(8),
    }
    for g, items in groups.items():
        t = time.time()
        vals = native.hper_batch([A for _, A in items], threads=threads)
        for (name, _), v in zip(items, vals):
            out[name] = str(v)
        print(g, f"{time.time() - t:.1f}s", flush=True)
    # cross-check one graph per group with the independent frontier DP
    for name, A in (("cubic24_seed0", W.config_n24()[0]), W.config_n60(0)[0]):
        assert int(out[name]) == per_dp(A), name
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
