#!/usr/bin/env python3
"""Batched allocator replay on one MI355X.

Workload (one step): the 4,096-heap batch -- 16 MiB arenas at 64 B
alignment, 100,000 requests per heap, sizes log-uniform on [64 B, 1 MiB],
alloc with probability 0.55, otherwise free a uniformly chosen live block --
replayed once with best fit and once with segregated fit: two persistent
launches of 409.6 M requests each, every heap's canonical final state dumped.
Inputs are synthetic (seeded) and resident in HBM before timing starts.

Printed: one JSON line with ops/s (value), the per-heap-launch baseline on a
sample of heaps, the replay kernel's roofline figures measured with HIP events
on its stream, the p50/p99 request latency of the device-resident service
under an open-loop load (100,000 clients, 1e7 requests/s offered), and the
CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("alloc+free ops/s on 1 MI355X (batched vs per-heap replay); "
          "p50/p99 req latency")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
# the service's stated latency bounds: p99 <= 200 us up to 1e7 requests/s,
# <= 1 ms at 2e7
P99_BOUND_US, P99_BOUND_RATE = 200.0, 1e7
P99_BOUND_TOP_US, P99_BOUND_TOP_RATE = 1000.0, 2e7
BYTES_PER_REQUEST = 16         # 8 B request read + 8 B result written
# MI355X instruction issue: 256 CUs x 4 SIMDs, 2.4 GHz; a wave64 VALU
# instruction takes 4 cycles on a 16-lane SIMD; one scalar unit per CU
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
SALU_ISSUE_PEAK = 256 * 2.4e9


def kernel_source_hash():
    """sha256 over the kernel sources and the device compiler flags: counter
    figures recorded for other sources or flags no longer describe the
    kernel being timed."""
    import hashlib
    from paper_2405_07079_amd import build as B
    d = os.path.join(ROOT, "paper_2405_07079_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    h.update(" ".join(B.FLAGS).encode())
    return h.hexdigest()


# The workload the committed summaries under profiles/ were taken on: heaps,
# requests per heap.  Their per-request figures are reported only for a run
# of the same workload.
PROFILED_WORKLOAD = (4096, 100_000)


def profiled_workload(heaps, requests):
    """True when a run replays the workload the committed summaries cover."""
    return (heaps, requests) == PROFILED_WORKLOAD


def recorded_traffic(algo_names):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, calibrated on a copy kernel), averaged over the timed
    launches; None when the summary is missing or was taken on other kernel
    sources."""
    path = os.path.join(ROOT, "profiles", "replay_4096x16MiB_hbm_traffic.txt")
    try:
        with open(path) as f:
            line = [x for x in f if x.startswith("machine-readable: ")][-1]
        rec = json.loads(line.split(": ", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    t = rec.get("traffic_bytes_per_launch", {})
    if not all(a in t for a in algo_names):
        return None
    return float(np.mean([t[a] for a in algo_names]))


def recorded_mix():
    """Per-request counts from the committed instruction-mix summary, while
    the kernel sources match: {algorithm: {"valu", "salu", "lds", "branch",
    "lds_conflict_cycles"}}; else None."""
    path = os.path.join(ROOT, "profiles", "replay_4096x16MiB_instruction_mix.txt")
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    if kernel_source_hash() not in text:
        return None
    mix = {}
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 8 and parts[0] in ("best_fit", "seg_fit"):
            v = [float(x) for x in parts[1:]]
            mix[parts[0]] = {"valu": v[0], "salu": v[1], "lds": v[2], "branch": v[3],
                             "lds_conflict_cycles": v[6]}
    return mix or None


def recorded_lds_conflicts():
    """LDS bank-conflict cycles per request (mean over the algorithms) from
    the committed instruction-mix summary, while the kernel sources match."""
    mix = recorded_mix()
    if not mix:
        return None
    return float(np.mean([m["lds_conflict_cycles"] for m in mix.values()]))


def issue_roofline(per_algo_ops):
    """Instruction issue against the chip's issue rates, from the recorded
    per-request counts and the measured requests/s: a wave64 VALU
    instruction holds a 16-lane SIMD for 4 cycles (1,024 SIMDs), and each
    CU's scalar unit issues one instruction per cycle (256 CUs), at
    2.4 GHz."""
    mix = recorded_mix()
    if not mix:
        return None
    out = {"bound": "issue", "unit": "G wave-instructions/s",
           "peak_valu": VALU_ISSUE_PEAK / 1e9, "peak_salu": SALU_ISSUE_PEAK / 1e9}
    for name, ops in per_algo_ops.items():
        if name not in mix:
            return None
        m = mix[name]
        out[name] = {"valu_per_request": m["valu"], "salu_per_request": m["salu"],
                     "valu_frac": m["valu"] * ops / VALU_ISSUE_PEAK,
                     "salu_frac": m["salu"] * ops / SALU_ISSUE_PEAK}
    return out


def bitmap_issue(ops):
    """The bitmask-allocator kernel's issue at `ops` requests/s, from the
    per-request counts in its committed instruction-mix summary while the
    kernel sources match; else None."""
    import re
    path = os.path.join(ROOT, "profiles", "bitmap_4096x16MiB_instruction_mix.txt")
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"^\s+VALU ([0-9.]+)\s+SALU ([0-9.]+)", text, re.M)
    if kernel_source_hash() not in text or not m:
        return None
    valu, salu = float(m.group(1)), float(m.group(2))
    return {"bound": "issue", "unit": "G wave-instructions/s",
            "peak_valu": VALU_ISSUE_PEAK / 1e9, "peak_salu": SALU_ISSUE_PEAK / 1e9,
            "valu_per_request": valu, "salu_per_request": salu,
            "valu_frac": valu * ops / VALU_ISSUE_PEAK, "salu_frac": salu * ops / SALU_ISSUE_PEAK}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def median_time(fn, runs=3):
    """Median wall time of `runs` calls of fn() (seconds)."""
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def event_ms(torch, stream, fn, runs):
    """Durations (ms) of `runs` calls of fn(), each bracketed by HIP events
    recorded on `stream` (the stream the work is enqueued on)."""
    evs = []
    for _ in range(runs):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def device_info(torch):
    """What the device reports about itself (torch's hipDeviceProp view)."""
    pr = torch.cuda.get_device_properties(0)
    out = {}
    for k in ("name", "gcnArchName", "multi_processor_count", "shared_memory_per_block",
              "L2_cache_size", "total_memory", "warp_size", "regs_per_multiprocessor"):
        v = getattr(pr, k, None)
        out[k] = v if isinstance(v, (int, float, str)) or v is None else str(v)
    return out


def host_info():
    """Host CPU model and the threads this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity": host_cores()}


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def paper_analog(W, torch):
    """The paper's comparison with the vendor's allocation calls, on this
    device: one stand-in trace (random allocations of 1 kB-16 MB and frees,
    5,000 steps) replayed call by call through hipMalloc / hipFree and
    through one of this library's segregated-fit heaps (4 GiB, 4 KiB
    granules; one kernel launch per call), each timed per call by a C++
    harness.  Fragmentation is 1 - in use / provisioned, where in use is the
    bytes the live requests asked for and provisioned is the device memory
    the process holds beyond its start (vendor; hipMemGetInfo) or the
    highest offset the heap has handed out (ours), averaged over the second
    half of the run."""
    import ctypes
    from paper_2405_07079_amd import build as hip_build
    A = ctypes.CDLL(hip_build.ANALOG)
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    A.hda_analog_vendor.restype = ctypes.c_int
    A.hda_analog_vendor.argtypes = [vp, i64, vp, vp, vp]
    A.hda_analog_heap.restype = ctypes.c_int
    A.hda_analog_heap.argtypes = [vp, i64, u64, u64, ctypes.c_int, ctypes.c_uint32, vp, vp]
    tb = W.paper_analog()
    req = np.ascontiguousarray(tb.req, np.int64)
    n = len(req)
    arena, align, algo = int(tb.arena[0]), int(tb.align[0]), int(tb.algo[0])

    def vendor(used=None):
        lat, res = np.zeros(n, np.int64), np.zeros(n, np.int64)
        rc = A.hda_analog_vendor(req.ctypes.data, n, lat.ctypes.data, res.ctypes.data,
                                 None if used is None else used.ctypes.data)
        if rc:
            raise RuntimeError(f"vendor replay failed: {rc}")
        return lat, res

    def ours():
        lat, res = np.zeros(n, np.int64), np.zeros(n, np.int64)
        rc = A.hda_analog_heap(req.ctypes.data, n, arena, align, algo, 8192,
                               lat.ctypes.data, res.ctypes.data)
        if rc:
            raise RuntimeError(f"heap replay failed: {rc}")
        return lat, res

    torch.cuda.synchronize()
    vendor()                                   # the first calls set up the runtime's pools
    vlat, vres = vendor()
    free0, total = torch.cuda.mem_get_info()
    used = np.zeros(n, np.int64)
    vendor(used)
    ours()
    olat, ores = ours()

    def in_use(res):
        live, cur, out = [], 0, np.zeros(n, np.int64)
        for i, q in enumerate(req.tolist()):
            if q >= 0 and res[i] >= 0:
                live.append(q)
                cur += q
            elif q < 0 and live:
                k = (((~q) & 0xFFFFFFFF) * len(live)) >> 32
                cur -= live[k]
                live[k] = live[-1]
                live.pop()
            out[i] = cur
        return out

    def lat_stats(lat, mask):
        x = lat[mask] / 1e3
        return float(np.percentile(x, 50)), float(np.percentile(x, 99)), float(x.max())

    def frag(use, prov):
        h = np.arange(n) >= n // 2
        ok = h & (prov > 0)
        return float(np.mean(1.0 - use[ok] / prov[ok]))

    allocs, frees = req >= 0, (req < 0) & (vlat > 0)
    v_use, o_use = in_use(vres), in_use(ores)
    v_prov = used - (total - free0)
    ends = np.where(allocs & (ores >= 0), ores + -(-req // align) * align, 0)
    o_prov = np.maximum.accumulate(ends)
    out = {"workload": f"{n} steps, alloc p={tb.meta['p_alloc']}, sizes log-uniform "
                       "1 KiB-16 MiB, frees of uniformly drawn live blocks; ours: one "
                       "segregated-fit heap of 4 GiB with 4 KiB granules, call by call"}
    for name, lat, use, prov, res in (("ours", olat, o_use, o_prov, ores),
                                      ("vendor", vlat, v_use, v_prov, vres)):
        a50, a99, amax = lat_stats(lat, allocs)
        f50, f99, fmax = lat_stats(lat, frees)
        out[name] = {"alloc_p50_us": a50, "alloc_p99_us": a99, "alloc_max_us": amax,
                     "free_p50_us": f50, "free_p99_us": f99, "free_max_us": fmax,
                     "allocs_failed": int((allocs & (res < 0)).sum()),
                     "peak_in_use_mib": float(use.max()) / 2**20,
                     "peak_provisioned_mib": float(prov.max()) / 2**20,
                     "fragmentation": frag(use, prov)}
    return out


# bytes the paper's own structures move per metadata touch: a free-list
# entry as (u32 address, u32 size) in granules; a segregated-fit record as
# address, size, prev_adj, next, prev and the free flag in u32 fields
ENTRY_BYTES, RECORD_BYTES = 8, 24


def oracle_metadata_bytes(stats, requests):
    """Metadata bytes per request the method itself touches, from the
    oracle's pinned counters (entries a fit search inspects, records the
    segregated-fit lists read or write)."""
    ex = float(stats[:, 0].sum())
    to = float(stats[:, 1].sum())
    return (ENTRY_BYTES * ex + RECORD_BYTES * to) / max(1, requests)


def leg_c1(W, hda, oracle, torch, stream):
    """One 64 KiB heap (16 B alignment), 10,000 requests, one wavefront:
    ns per request for every algorithm (first fit is the configuration as
    stated; the others run the same trace)."""
    base = W.single_heap()
    out = {"workload": "1 heap, 64 KiB arena, 16 B alignment, 10,000 requests (alloc p=0.6, "
                       "sizes log-uniform 16 B-4 KiB), one wavefront per launch",
           "unit": "ns/request", "per_algorithm": {}, "cpu_baseline": {}}
    for algo in range(5):
        b = base.with_algo(algo)
        db = hda.upload(b)
        hda.hda_replay(db, stream)
        torch.cuda.synchronize()
        if int((db.status != 0).sum().item()):
            raise RuntimeError("single-heap leg: heap reported an error")
        ms = float(np.median(event_ms(torch, stream, lambda: hda.hda_replay(db, stream), 7)))
        name = W.ALGO_NAMES[algo]
        out["per_algorithm"][name] = ms * 1e6 / b.requests
        req = np.ascontiguousarray(b.req)
        ct = median_time(lambda: oracle.replay_heap(algo, int(b.arena[0]), int(b.align[0]), req))
        out["cpu_baseline"][name] = ct * 1e9 / b.requests
        del db
    out["value"] = out["per_algorithm"]["first_fit"]
    out["cpu_baseline"].update({"unit": "ns/request", "cores": 1, "kind": "oracle",
                                "sample": "the whole trace, median of 3"})
    return out


def leg_c3(W, hda, oracle, torch, stream, cores):
    """The uneven batch (16,384 heaps, arenas 1 MiB-1 GiB, Pareto trace
    lengths, four algorithms) in longest-first order: default tuning, the
    autotuner's choice, and that choice launched as a captured graph;
    per-heap launches on a sample."""
    t0 = time.perf_counter()
    b = W.uneven_batch()
    log(f"[bench] c3: generated {b.requests} requests in {time.perf_counter() - t0:.1f} s")
    db = hda.upload(b)
    run = lambda: hda.hda_replay(db, stream)  # noqa: E731
    run()
    torch.cuda.synchronize()
    default_ms = float(np.median(event_ms(torch, stream, run, 3)))
    t0 = time.perf_counter()
    tune = hda.hda_replay_autotune(db, 0, stream)
    tune_s = time.perf_counter() - t0
    hda.retune(db, tune)
    run()
    torch.cuda.synchronize()
    tuned_ms = float(np.median(event_ms(torch, stream, run, 3)))
    g = hda.ReplayGraph(db)
    try:
        g.launch(stream)
        torch.cuda.synchronize()
        graph_ms = float(np.median(event_ms(torch, stream, lambda: g.launch(stream), 3)))
    finally:
        g.close()
    if int((db.status != 0).sum().item()):
        raise RuntimeError("uneven-batch leg: heaps reported errors")
    resolved = hda.hda_replay_resolve(db)
    del db
    # one launch per heap on a sample of 256 heaps (every 64th heap)
    idx = np.arange(0, b.heaps, 64)
    sub = b.subset(idx)
    sdb = hda.upload(sub)
    hda.hda_replay_per_heap(sdb, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hda.hda_replay_per_heap(sdb, stream)
    torch.cuda.synchronize()
    ph = sub.requests / (time.perf_counter() - t1)
    del sdb
    ct = median_time(lambda: oracle.replay_batch(b, threads=cores, want_state=False))
    ops = lambda ms: b.requests / (ms / 1e3)  # noqa: E731
    return {"workload": f"{b.heaps} heaps, arenas log-uniform 1 MiB-1 GiB (32 B alignment), "
                        f"trace lengths Pareto(1.5) clipped to 1k-1M ({b.requests} requests), "
                        "first/next/best/segregated fit uniformly, longest first",
            "unit": "ops/s", "value": ops(graph_ms),
            "default": {"ms": default_ms, "ops_s": ops(default_ms)},
            "autotuned": {"ms": tuned_ms, "ops_s": ops(tuned_ms), "tuning": resolved,
                          "autotune_s": tune_s},
            "autotuned_graph": {"ms": graph_ms, "ops_s": ops(graph_ms)},
            "per_heap_launch": {"value": ph, "unit": "ops/s",
                                "sample": f"{sub.heaps} heaps (every 64th), {sub.requests} "
                                          "requests, one launch per heap"},
            "cpu_baseline": {"value": b.requests / ct, "unit": "ops/s", "cores": cores,
                             "kind": "oracle",
                             "sample": f"the whole batch, median of 3 ({ct:.1f} s)"}}


def leg_c5(W, hda, oracle, torch, stream):
    """The 256 GiB segregated-fit heap (4 KiB granules), 50 M requests, on
    the ordered core (one wavefront with the whole LDS of a workgroup)."""
    import hashlib
    t0 = time.perf_counter()
    b = W.large_seg_fit()
    log(f"[bench] c5: generated {b.requests} requests in {time.perf_counter() - t0:.1f} s")
    tu = hda.tuning(heavy_heaps=1, heavy_kib=158)
    db = hda.upload(b, tuning=tu, meta_free=4096, meta_live=16384)
    ms = event_ms(torch, stream, lambda: hda.hda_replay(db, stream), 1)[0]
    status = int(db.status[0].item())
    if status:
        raise RuntimeError(f"256 GiB leg: status {status}")
    digest_ok = None
    gp = os.path.join(ROOT, "tests", "golden", "large_seg_fit_256GiB.json")
    if os.path.exists(gp):
        with open(gp) as f:
            g = json.load(f)
        res = db.res.cpu().numpy()
        digest_ok = hashlib.sha256(np.ascontiguousarray(res, "<i8").tobytes()).hexdigest() == \
            g["results_sha256"]
    resolved = hda.hda_replay_resolve(db)
    del db
    n = 2_000_000
    req = np.ascontiguousarray(b.req[:n])
    ct = median_time(lambda: oracle.replay_heap(W.SEG_FIT, int(b.arena[0]), int(b.align[0]), req))
    return {"workload": "1 heap, 256 GiB virtual arena, 4 KiB granules, segregated fit, 50 M "
                        "requests (alloc p=0.5, sizes geometric over the 4 KiB-64 MiB classes), "
                        "replayed in order by one wavefront",
            "unit": "ops/s", "value": b.requests / (ms / 1e3), "ms": ms,
            "ns_per_request": ms * 1e6 / b.requests, "tuning": resolved,
            "results_equal_oracle_digest": digest_ok,
            "cpu_baseline": {"value": n / ct, "unit": "ops/s", "cores": 1, "kind": "oracle",
                             "sample": f"the first {n} requests, median of 3"}}


def leg_serving(hda, rates, clients, seconds, bound_us, bound_rate):
    """The device-resident service under open-loop Poisson load from
    `clients` clients (one heap each) at each rate: throughput and latency
    percentiles from arrival to completion."""
    srv = hda.Server(max_heaps=clients + 16, max_seconds=600)
    by_rate = []
    try:
        for rate in rates:
            rep, _ = srv.load(clients=clients, rate=rate, warmup_s=0.5, measure_s=seconds,
                              threads=max(1, min(16, host_cores())))
            if rep["errors"]:
                raise RuntimeError(f"serving leg reported {rep['errors']} errors at {rate:g}/s")
            by_rate.append({"offered_rate": rate, "throughput": rep["throughput"],
                            "p50_us": rep["p50_us"], "p90_us": rep["p90_us"],
                            "p99_us": rep["p99_us"], "p999_us": rep["p999_us"],
                            "max_us": rep["max_us"], "completed": rep["completed"],
                            "alloc_fail": rep["alloc_fail"], "window_s": rep["window_s"],
                            "components_us": {
                                k: {"p50": rep[f"{k}_p50_us"], "p99": rep[f"{k}_p99_us"]}
                                for k in ("host", "queue", "service", "transit")}})
            log(f"[bench] serving at {rate:.3g}/s: {rep['throughput']:.3g}/s, "
                f"p50 {rep['p50_us']:.1f} us, p99 {rep['p99_us']:.1f} us; p99 of host "
                f"{rep['host_p99_us']:.1f}, queue {rep['queue_p99_us']:.1f}, service "
                f"{rep['service_p99_us']:.1f}, transit {rep['transit_p99_us']:.1f} us")
    finally:
        srv.stop()
    within = [r["p99_us"] <= (bound_us if r["offered_rate"] <= bound_rate else P99_BOUND_TOP_US)
              for r in by_rate if r["offered_rate"] <= P99_BOUND_TOP_RATE]
    return {"clients": clients, "unit": "requests/s",
            "p99_bound_us": {f"{bound_rate:g}": bound_us,
                             f"{P99_BOUND_TOP_RATE:g}": P99_BOUND_TOP_US},
            "within_bound": bool(within) and all(within), "by_rate": by_rate}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--heaps", type=int, default=4096)
    ap.add_argument("--requests", type=int, default=100_000)
    ap.add_argument("--per-heap-sample", type=int, default=64,
                    help="heaps per algorithm replayed one launch per heap")
    ap.add_argument("--cpu-sample", type=int, default=1024,
                    help="heaps per algorithm replayed by the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-rates", type=str, default="1e6,2e6,5e6,1e7,2e7",
                    help="serving leg: open-loop arrival rates per second, comma-separated "
                         "(empty or 0 = skip)")
    ap.add_argument("--serve-clients", type=int, default=100_000)
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="serving leg: measured window (after 0.5 s of warmup)")
    ap.add_argument("--tuning", type=str, default="0,0,0,0,0,0",
                    help="heaps_per_group,reg_free,reg_live,lds_free,lds_live,groups "
                         "(0 = default, -1 = none)")
    ap.add_argument("--no-paper-analog", action="store_true",
                    help="skip the per-call comparison with hipMalloc / hipFree")
    ap.add_argument("--no-bitmap", action="store_true",
                    help="skip the leg that replays the batch with the bitmask allocator")
    ap.add_argument("--no-tlsf", action="store_true",
                    help="skip the leg that replays the batch with two-level segregated fit")
    ap.add_argument("--partial-frees", type=float, default=0.02,
                    help="fraction of frees that are partial (Alg. 2) in the partial-"
                         "deallocation leg, a best-fit batch of the same shape (0: skip)")
    ap.add_argument("--no-c1", action="store_true",
                    help="skip the single 64 KiB heap leg")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the uneven-batch leg (16,384 heaps)")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the 256 GiB single-heap leg (50 M requests)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (a kernel of "
                         "known traffic for scaling memory counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the replay runs on exactly one GPU (asked for {args.gpus}); "
              "heaps are independent, so N GPUs would each replay their own share "
              "with no communication -- run N=1.", file=sys.stderr)
        return 2
    profiled = profiled_workload(args.heaps, args.requests)

    import torch
    from paper_2405_07079_amd import hda
    from paper_2405_07079_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    tuning = tuple(int(x) for x in args.tuning.split(","))
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {n} bytes done")
        del src, dst

    t0 = time.perf_counter()
    batch = W.uniform_batch(heaps=args.heaps, n=args.requests)
    log(f"[bench] generated {batch.requests} requests in {time.perf_counter() - t0:.1f} s")
    algos = (W.BEST_FIT, W.SEG_FIT)
    dbs = {}
    for algo in algos:
        dbs[algo] = hda.upload(batch.with_algo(algo), tuning=tuning,
                               share=dbs.get(algos[0]))
    torch.cuda.synchronize()
    resolved = hda.hda_replay_resolve(dbs[algos[0]])
    log(f"[bench] uploaded; tuning {resolved}")

    stream = torch.cuda.current_stream()
    per_launch_ms = {a: [] for a in algos}

    def step(record):
        for algo in algos:
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            hda.hda_replay(dbs[algo], stream)
            if record:
                e1.record(stream)
                per_launch_ms[algo].append((e0, e1))

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    for algo in algos:
        st = dbs[algo].status
        if int((st != 0).sum().item()):
            raise RuntimeError(f"heaps reported errors: {st.unique().tolist()}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] {args.steps} timed steps in {elapsed:.3f} s")

    ops_per_step = batch.requests * len(algos)
    value = ops_per_step * args.steps / elapsed
    launch_ms = {a: [x[0].elapsed_time(x[1]) for x in per_launch_ms[a]] for a in algos}
    per_algo = {W.ALGO_NAMES[a]: batch.requests / (np.mean(launch_ms[a]) / 1e3) for a in algos}
    all_ms = [m for a in algos for m in launch_ms[a]]
    avg_launch_s = float(np.mean(all_ms)) / 1e3
    achieved = BYTES_PER_REQUEST * batch.requests / avg_launch_s / 1e9

    # per-heap-launch baseline: the same kernel body, one launch per heap
    S = min(args.per_heap_sample, batch.heaps)
    sub = batch.subset(np.arange(S))
    ph_ops = 0
    ph_time = 0.0
    for algo in algos:
        db = hda.upload(sub.with_algo(algo), tuning=tuning)
        hda.hda_replay_per_heap(db, stream)           # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hda.hda_replay_per_heap(db, stream)
        torch.cuda.synchronize()
        ph_time += time.perf_counter() - t1
        ph_ops += sub.requests
        del db
    per_heap_value = ph_ops / ph_time
    log(f"[bench] per-heap launches: {per_heap_value / 1e6:.2f} M ops/s on {S} heaps/algo")

    tlsf = None
    if not args.no_tlsf:
        # the same batch replayed with two-level segregated fit (Sec. V-B)
        tdb = hda.upload(batch.with_algo(W.TLSF), tuning=tuning, share=dbs[algos[0]])
        hda.hda_replay(tdb, stream)
        torch.cuda.synchronize()
        if int((tdb.status != 0).sum().item()):
            raise RuntimeError("TLSF leg: heaps reported errors")
        tms = []
        for _ in range(max(1, args.steps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            hda.hda_replay(tdb, stream)
            e1.record(stream)
            tms.append((e0, e1))
        torch.cuda.synchronize()
        tms = [a.elapsed_time(b) for a, b in tms]
        tlsf = {"workload": f"the batch above replayed with two-level segregated fit "
                            f"(32 sub-classes per power of two)",
                "value": batch.requests / (float(np.median(tms)) / 1e3), "unit": "ops/s",
                "launch_ms": float(np.median(tms))}
        del tdb
        log(f"[bench] tlsf: {tlsf['value'] / 1e9:.3f} G ops/s")

    bitmap = None
    if not args.no_bitmap:
        # the same batch replayed by the bitmask allocator (Sec. III-B): one
        # flag per granule, next-fit scan, its own kernel
        bb = batch.with_algo(W.BITMAP)
        bdb = hda.upload(bb, share=dbs[algos[0]])
        mg = hda.max_granules(bb)
        hda.hda_bitmap_replay(bdb, mg, stream)
        torch.cuda.synchronize()
        if int((bdb.status != 0).sum().item()):
            raise RuntimeError("bitmap leg: heaps reported errors")
        bms = []
        for _ in range(max(1, min(args.steps, 3))):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            hda.hda_bitmap_replay(bdb, mg, stream)
            e1.record(stream)
            bms.append((e0, e1))
        torch.cuda.synchronize()
        bms = [a.elapsed_time(b) for a, b in bms]
        bitmap = {"workload": "the batch above replayed by the bitmask allocator (one flag "
                              "per granule, 32 KiB per heap, and a run summary per 4,096 "
                              "granules; next-fit search from the rover)",
                  "value": batch.requests / (float(np.median(bms)) / 1e3), "unit": "ops/s",
                  "launch_ms": float(np.median(bms))}
        bitmap["issue"] = (bitmap_issue(bitmap["value"]) if profiled else None)
        del bdb
        log(f"[bench] bitmap: {bitmap['value'] / 1e9:.3f} G ops/s")

    partial = None
    if args.partial_frees > 0:
        # the same batch shape on best fit, with that fraction of the frees
        # partial: the victim keeps a uniform fraction of its granules
        pb = W.uniform_batch(heaps=args.heaps, n=args.requests, algo=W.BEST_FIT,
                             p_partial=args.partial_frees)
        pdb = hda.upload(pb, tuning=tuning)
        hda.hda_replay(pdb, stream)
        torch.cuda.synchronize()
        if int((pdb.status != 0).sum().item()):
            raise RuntimeError("partial-free leg: heaps reported errors")
        pms = []
        for _ in range(max(1, args.steps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            hda.hda_replay(pdb, stream)
            e1.record(stream)
            pms.append((e0, e1))
        torch.cuda.synchronize()
        pms = [a.elapsed_time(b) for a, b in pms]
        n_partial = int((pb.req < -(1 << 32)).sum())
        partial = {"workload": f"{pb.heaps} heaps x 16 MiB, {args.requests} requests each, "
                               f"best fit, {args.partial_frees:g} of the frees partial",
                   "value": pb.requests / (float(np.median(pms)) / 1e3), "unit": "ops/s",
                   "launch_ms": float(np.median(pms)), "partial_frees": n_partial,
                   "frees": int((pb.req < 0).sum())}
        del pdb
        log(f"[bench] partial frees ({args.partial_frees:g}): "
            f"{partial['value'] / 1e9:.3f} G ops/s")

    serving = None
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip() and float(x) > 0]
    if rates:
        # device-resident service: one heap per client (64 MiB-4 GiB, 512 B
        # alignment, segregated fit), Poisson arrivals, 70 % power-of-two sizes
        # 512 B-256 MiB and 30 % log-uniform, exponential lifetimes (mean 500
        # requests); latency from arrival to completion seen by the client
        serving = leg_serving(hda, rates, args.serve_clients, args.serve_seconds,
                              P99_BOUND_US, P99_BOUND_RATE)

    analog = None
    if not args.no_paper_analog:
        analog = paper_analog(W, torch)
        log(f"[bench] paper analog: ours alloc p50 {analog['ours']['alloc_p50_us']:.1f} us, "
            f"hipMalloc p50 {analog['vendor']['alloc_p50_us']:.1f} us")

    cpu = None
    meta_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        cores = host_cores()
        C = min(args.cpu_sample, batch.heaps)
        csub = batch.subset(np.arange(C))
        ct = median_time(lambda: [oracle.replay_batch(csub.with_algo(a), threads=cores,
                                                      want_state=True) for a in algos])
        # the method's own metadata bytes per request, from the oracle's
        # pinned counters on the same sample
        meta_oracle = {}
        for a in algos:
            _, _, st = oracle.replay_batch(csub.with_algo(a), threads=cores, want_state=False,
                                           want_stats=True)
            meta_oracle[W.ALGO_NAMES[a]] = oracle_metadata_bytes(st, csub.requests)
        one = batch.subset(np.arange(min(16, C)))
        c1t = median_time(lambda: [oracle.replay_batch(one.with_algo(a), threads=1,
                                                       want_state=True) for a in algos])
        cpu = {"value": csub.requests * len(algos) / ct, "unit": "ops/s", "cores": cores,
               "value_1_thread": one.requests * len(algos) / c1t,
               "kind": "oracle",
               "sample": f"first {C} heaps of the batch x (best fit, seg fit), "
                         f"{csub.requests * len(algos)} requests, median of 3 "
                         f"({ct:.1f} s wall on {cores} threads)"}
        log(f"[bench] cpu oracle: {cpu['value'] / 1e6:.2f} M ops/s on {cores} threads")
        small = batch.subset(np.arange(min(256, batch.heaps)))
        for leg, sb in ((bitmap, small.with_algo(W.BITMAP)), (tlsf, small.with_algo(W.TLSF)),
                        (partial, None if partial is None else
                         pb.subset(np.arange(min(256, pb.heaps))))):
            if leg is None:
                continue
            t = median_time(lambda: oracle.replay_batch(sb, threads=cores, want_state=True))
            leg["cpu_baseline"] = {"value": sb.requests / t, "unit": "ops/s", "cores": cores,
                                   "kind": "oracle",
                                   "sample": f"first {sb.heaps} heaps, {sb.requests} "
                                             f"requests, median of 3"}

    import oracle as _oracle
    c1 = None if args.no_c1 else leg_c1(W, hda, _oracle, torch, stream)
    if c1:
        log(f"[bench] c1: {c1['per_algorithm']}")
    c3 = None if args.no_c3 else leg_c3(W, hda, _oracle, torch, stream, host_cores())
    if c3:
        log(f"[bench] c3: default {c3['default']['ops_s'] / 1e6:.1f} M, autotuned "
            f"{c3['autotuned']['ops_s'] / 1e6:.1f} M, graph {c3['value'] / 1e6:.1f} M ops/s")
    c5 = None if args.no_c5 else leg_c5(W, hda, _oracle, torch, stream)
    if c5:
        log(f"[bench] c5: {c5['value'] / 1e6:.2f} M ops/s ({c5['ms'] / 1e3:.1f} s)")

    traffic = recorded_traffic([W.ALGO_NAMES[a] for a in algos]) if profiled else None
    state_bytes = float(np.mean([int(dbs[a].state_len.sum().item()) * 8 for a in algos]))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{batch.heaps} heaps x 16 MiB arena, 64 B alignment, "
                        f"{args.requests} requests each, sizes log-uniform 64 B-1 MiB, "
                        "alloc p=0.55; best fit and segregated fit, one persistent "
                        "launch each, one wavefront per heap",
            "heaps": batch.heaps,
            "requests_per_step": ops_per_step,
            "tuning": resolved,
        },
        "per_algorithm_ops_s": per_algo,
        "per_heap_launch": {"value": per_heap_value, "unit": "ops/s",
                            "sample": f"first {S} heaps x (best fit, seg fit), "
                                      "one launch per heap",
                            "batched_speedup": value / per_heap_value},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch",
                     "traffic_frac": (None if traffic is None else
                                      traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS),
                     # HBM bytes beyond the requests, results and state dumps
                     "metadata_hbm_bytes_per_request": (
                         None if traffic is None else
                         max(0.0, (traffic - BYTES_PER_REQUEST * batch.requests
                                   - state_bytes) / batch.requests)),
                     # what the method's own structures would touch per request
                     # (oracle counters; 8 B per list entry, 24 B per record)
                     "metadata_bytes_per_request_oracle": meta_oracle,
                     "lds_bank_conflict_cycles_per_request": (
                         recorded_lds_conflicts() if profiled else None),
                     # what bounds this kernel: instruction issue
                     "issue": issue_roofline(per_algo) if profiled else None,
                     "kernel": f"lean_kernel<{max(resolved['reg_free'], 0)}>",
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "bytes_per_request": BYTES_PER_REQUEST,
                     "requests_per_launch": batch.requests},
        "tlsf": tlsf,
        "bitmap": bitmap,
        "partial_free": partial,
        "paper_analog": analog,
        "serving": serving,
        "c1": c1,
        "c3": c3,
        "c5": c5,
        "device": device_info(torch),
        "host": host_info(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
