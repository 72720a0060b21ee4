"""Write the stored expected values under tests/golden/ from the CPU oracle.

Only the oracle and the seeded input generator are called here.  Run from the
repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2405_07079_amd import workloads as W  # noqa: E402


def digest(a):
    return hashlib.sha256(a.astype("<i8").tobytes()).hexdigest()


def single_heap_fixture():
    b = W.single_heap()
    out = dict(workload="single heap, 64 KiB arena, 16 B alignment, 10,000 "
                        "requests, seed 1 (alloc w.p. 0.6, log-uniform 16 B-4 KiB)",
               trace_sha256=digest(b.req), algos={})
    for algo, name in W.ALGO_NAMES.items():
        res, st = oracle.replay_heap(algo, int(b.arena[0]), int(b.align[0]), b.req)
        out["algos"][name] = dict(
            results_sha256=digest(res), state_sha256=digest(st),
            allocs_ok=int(((b.req >= 0) & (res >= 0)).sum()),
            allocs_failed=int(((b.req >= 0) & (res < 0)).sum()),
            first_results=[int(x) for x in res[:24]],
            final_free_blocks=int(st[0]))
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "single_heap_64KiB.json"), "w") as f:
        json.dump(single_heap_fixture(), f, indent=1)
        f.write("\n")
    print("wrote", os.path.join(HERE, "single_heap_64KiB.json"))
