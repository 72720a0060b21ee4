"""Host-side pieces of bench.py: the issue figures it derives from the
committed instruction-mix summaries, and the one-GPU rule.  No GPU
involved."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions/s: 1,024 SIMDs, 4 cycles each


def test_issue_peaks():
    assert bench.VALU_ISSUE_PEAK == pytest.approx(PEAK)
    assert bench.SALU_ISSUE_PEAK == pytest.approx(256 * 2.4e9)


def profile_matches(name):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        return bench.kernel_source_hash() in f.read()


def test_bitmap_issue_from_profile():
    r = bench.bitmap_issue(2e9)
    if not profile_matches("bitmap_4096x16MiB_instruction_mix.txt"):
        assert r is None          # figures of other sources are not reported
        return
    assert r["valu_per_request"] > 0 and r["salu_per_request"] > 0
    assert r["valu_frac"] == pytest.approx(r["valu_per_request"] * 2e9 / PEAK)
    assert r["salu_frac"] == pytest.approx(r["salu_per_request"] * 2e9 / (256 * 2.4e9))


def test_replay_issue_from_profile():
    r = bench.issue_roofline({"best_fit": 5e9, "seg_fit": 4e9})
    if not profile_matches("replay_4096x16MiB_instruction_mix.txt"):
        assert r is None
        return
    for name, ops in (("best_fit", 5e9), ("seg_fit", 4e9)):
        m = r[name]
        assert m["valu_frac"] == pytest.approx(m["valu_per_request"] * ops / PEAK)


def test_profile_figures_only_for_the_profiled_workload():
    """The per-request counts and traffic of the committed summaries are
    reported only for a run of the workload they were taken on, which each
    summary's header names."""
    heaps, requests = bench.PROFILED_WORKLOAD
    assert bench.profiled_workload(heaps, requests)
    assert not bench.profiled_workload(heaps, requests // 5)
    assert not bench.profiled_workload(64, requests)
    named = f"{heaps} heaps x {requests:,} requests"
    for name in ("bitmap_4096x16MiB_instruction_mix.txt",
                 "replay_4096x16MiB_instruction_mix.txt",
                 "replay_4096x16MiB_hbm_traffic.txt",
                 "replay_4096x16MiB_kernel_trace.txt"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            head = " ".join(f.read().split("\n")[:3])
        assert named in head, name


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode != 0
    assert "exactly one GPU" in p.stdout + p.stderr
