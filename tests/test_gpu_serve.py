"""The device-resident allocator service against the oracle: results of
interleaved clients, the open-loop load's logged clients, a client alone vs
in the mix, admission by metadata budget, and the watchdog."""
import time

import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda

pytestmark = pytest.mark.gpu
pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture
def server():
    s = hda.Server(max_heaps=256, waves=16, max_seconds=120)
    yield s
    s.stop()


def test_interleaved_heaps_match_oracle(server):
    say("case: 8 heaps (all five algorithms), interleaved async submits")
    rng = np.random.default_rng(3)
    heaps, models, live = [], [], []
    for k in range(8):
        algo = k % 5                  # every algorithm, TLSF included
        A = int(rng.integers(64, 4096)) * 256
        heaps.append(server.open(A, 256, algo))
        models.append(oracle.Heap(algo, A, 256))
        live.append([])
    for rnd in range(60):
        tickets = []
        for k in range(8):            # one request per heap per round, all in flight
            if live[k] and rng.random() < 0.45:
                x = live[k].pop(int(rng.integers(len(live[k]))))
                tickets.append((k, hda.HDA_OP_FREE, x, server.submit(heaps[k], hda.HDA_OP_FREE, x)))
            else:
                size = int(rng.integers(0, 60_000))
                tickets.append((k, hda.HDA_OP_ALLOC, size,
                                server.submit(heaps[k], hda.HDA_OP_ALLOC, size)))
        for k, op, arg, t in tickets:
            r = server.wait(t)
            if op == hda.HDA_OP_ALLOC:
                assert r == models[k].alloc(arg), (rnd, k)
                if r >= 0:
                    live[k].append(r)
            else:
                assert r == models[k].free(arg) == 0
    # bad frees are rejected and change nothing
    assert server.free(heaps[0], 7) == hda.HDA_E_BADFREE
    for h in heaps:
        server.close_heap(h)


def replay_log(log):
    """Replay one logged client on an oracle heap; returns the oracle results."""
    _, arena, align = (int(x) for x in log[0])
    h = oracle.Heap(hda.SEG_FIT, arena, align)
    out = []
    for op, arg, _ in log[1:]:
        out.append(h.alloc(int(arg)) if op == hda.HDA_OP_ALLOC else h.free(int(arg)))
    return np.array(out, np.int64)


def test_load_results_match_oracle_and_alone(server):
    say("case: open-loop load, 96 clients, logged")
    rep, logs = server.load(clients=96, rate=20_000, warmup_s=0.2, measure_s=0.8,
                            log_clients=96, log_cap=4096, arena=(1 << 20, 64 << 20),
                            size=(512, 4 << 20), pow2=(9, 22), lifetime_mean=50)
    say("report", rep)
    assert rep["errors"] == 0 and rep["completed"] == rep["issued"] > 1000
    assert rep["alloc_ok"] > 0 and rep["frees"] > 0
    for c, log in enumerate(logs):
        assert len(log) > 1
        assert np.array_equal(log[1:, 2], replay_log(log)), f"client {c}"
    # client 0 alone: the same requests on a fresh heap, one at a time
    _, arena, align = (int(x) for x in logs[0][0])
    h = server.open(arena, align, hda.SEG_FIT)
    alone = [server.wait(server.submit(h, int(op), int(arg))) for op, arg, _ in logs[0][1:]]
    assert np.array_equal(np.array(alone), logs[0][1:, 2])
    server.close_heap(h)


def test_admission_by_metadata_budget():
    say("case: admission budget")
    # a slot with 64 free and 64 live entries: 320 B of registers and counts,
    # 12 B per free entry, 8 B per live entry, rounded to 256 B
    slot = (320 + 64 * 12 + 64 * 8 + 255) // 256 * 256
    s = hda.Server(max_heaps=16, waves=4, slot_free=64, slot_live=64, max_seconds=60,
                   meta_budget=3 * slot)
    try:
        a = [s.open(1 << 20, 64, hda.SEG_FIT) for _ in range(3)]
        with pytest.raises(hda.HdaError) as e:
            s.open(1 << 20, 64, hda.SEG_FIT)
        assert e.value.code == hda.HDA_E_NOMETA
        assert s.alloc(a[0], 1000) == 0
        s.close_heap(a[1])              # releases its share of the budget
        b = s.open(1 << 20, 64, hda.SEG_FIT)
        assert s.alloc(b, 100) == 0
    finally:
        s.stop()


def split_sessions(log):
    """A logged client's sessions: lists of rows, each starting with its
    (0, arena, align) row."""
    starts = [i for i in range(len(log)) if log[i, 0] == 0] + [len(log)]
    return [log[a:b] for a, b in zip(starts, starts[1:])]


def test_admission_under_load_with_sessions():
    """2,000 clients under open-loop load with a metadata budget of 200 heaps
    (10 % of what holding every client's heap would need).  Clients work in
    sessions of 40 requests: a session opens a heap when the budget admits
    it and closes it at the end, so closed sessions make room for waiting
    clients while the others' requests are on the GPU.  Every logged
    session's results equal an oracle replay of that session, and one of
    them replayed alone gives the same results as in the mix."""
    slot = hda.Server.slot_bytes(64, 64)
    clients, admitted = 2000, 200
    s = hda.Server(max_heaps=clients, waves=32, slot_free=64, slot_live=64, max_seconds=120,
                   meta_budget=admitted * slot)
    try:
        say(f"case: admission under load, {clients} clients, budget {admitted} heaps")
        rep, logs = s.load(clients=clients, rate=200_000, warmup_s=0.2, measure_s=1.0,
                           threads=4, session_len=40, log_clients=60, log_cap=8192,
                           arena=(1 << 20, 64 << 20), size=(512, 1 << 20), pow2=(9, 20),
                           lifetime_mean=15)
        say("report", rep)
        assert rep["errors"] == 0 and rep["completed"] == rep["issued"] > 100_000
        assert rep["slot_bytes"] == slot
        assert admitted // 2 < rep["max_open"] <= admitted
        assert rep["sessions"] > clients          # budget freed and re-used
        assert rep["admission_waits"] > 0
        n_sessions = 0
        for c, log in enumerate(logs):
            for sess in split_sessions(log):
                if len(sess) > 1:
                    assert np.array_equal(sess[1:, 2], replay_log(sess)), f"client {c}"
                    n_sessions += 1
        assert n_sessions > len(logs)
        # one session alone on a fresh heap: the same results as in the mix
        sess = max((x for lg in logs for x in split_sessions(lg)), key=len)
        _, arena, align = (int(x) for x in sess[0])
        h = s.open(arena, align, hda.SEG_FIT)
        alone = [s.wait(s.submit(h, int(op), int(arg))) for op, arg, _ in sess[1:]]
        assert np.array_equal(np.array(alone), sess[1:, 2])
        s.close_heap(h)
    finally:
        s.stop()


def test_watchdog_ends_the_kernel():
    say("case: watchdog")
    s = hda.Server(max_heaps=4, waves=2, max_seconds=1.0)
    h = s.open(1 << 20, 64, hda.FIRST_FIT)
    assert s.alloc(h, 64) == 0
    time.sleep(2.0)
    t = time.time()
    s.stop()                       # the kernel has already left its loop
    assert time.time() - t < 5.0
