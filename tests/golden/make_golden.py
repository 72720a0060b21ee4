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


def large_seg_fit_fixture(samples=4096):
    """The 256 GiB segregated-fit heap at full length: digests of all 50 M
    results and of the final state, the table sizes, and results at seeded
    sample positions (for a check that does not need the full output)."""
    import numpy as np
    b = W.large_seg_fit()
    res, st = oracle.replay_heap(W.SEG_FIT, int(b.arena[0]), int(b.align[0]), b.req)
    pos = np.sort(np.random.default_rng(55).choice(len(res), samples, replace=False))
    parsed = oracle.parse_state(st, W.SEG_FIT)
    return dict(workload="one 256 GiB heap, 4 KiB granularity, segregated fit, "
                         "50,000,000 requests, seed 5 (alloc w.p. 0.5, sizes geometric "
                         "over the 4 KiB-64 MiB classes)",
                trace_sha256=digest(b.req), results_sha256=digest(res),
                state_sha256=digest(st), final_free_blocks=len(parsed["free"]),
                final_live_blocks=len(parsed["live"]),
                allocs_failed=int(((b.req >= 0) & (res < 0)).sum()),
                sample_positions=[int(x) for x in pos],
                sample_results=[int(x) for x in res[pos]])


def write(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    print("wrote", os.path.join(HERE, name))


if __name__ == "__main__":
    which = sys.argv[1:] or ["single"]
    if "single" in which:
        write("single_heap_64KiB.json", single_heap_fixture())
    if "large" in which:
        write("large_seg_fit_256GiB.json", large_seg_fit_fixture())
