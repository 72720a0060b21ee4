"""Call-by-call heaps on the GPU (hda_heap_create / hda_alloc / hda_free /
hda_heap_state) against oracle heaps driven with the same calls."""
import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda

pytestmark = pytest.mark.gpu
pytest.importorskip("torch")


@pytest.mark.parametrize("algo", (0, 1, 2, 3, 4))
def test_calls_match_oracle(algo):
    print(f"case: call-by-call heap algo {algo}", flush=True)
    A, g = 1 << 16, 32
    gh = hda.Heap(A, g, algo, meta_cap=512)
    oh = oracle.Heap(algo, A, g)
    rng = np.random.default_rng(algo)
    live = []
    for step in range(300):
        if live and rng.random() < 0.45:
            x = live.pop(int(rng.integers(len(live))))
            assert gh.free(x) == oh.free(x) == 0
        else:
            size = int(rng.integers(0, 3000))
            r = gh.alloc(size)
            assert r == oh.alloc(size), step
            if r >= 0:
                live.append(r)
        if step % 50 == 0:
            assert np.array_equal(gh.state(), oh.state())
    assert np.array_equal(gh.state(), oh.state())
    gh.close()


@pytest.mark.parametrize("algo", (0, 1, 2, 3, 4))
def test_arena_of_2_32_minus_1_granules(algo):
    """The largest arena a heap may have: the whole free arena's size and the
    end of its last block are both 2^32 - 1 granules."""
    print(f"case: 2^32 - 1 granule heap algo {algo}", flush=True)
    g = 64
    A = ((1 << 32) - 1) * g
    gh = hda.Heap(A, g, algo, meta_cap=64)
    oh = oracle.Heap(algo, A, g)
    whole = gh.alloc(A)
    assert whole == oh.alloc(A)
    if whole >= 0:
        assert gh.free(whole) == oh.free(whole) == 0
    lo = gh.alloc(((1 << 31) - 1) * g)
    hi = gh.alloc((1 << 31) * g)
    assert (lo, hi) == (oh.alloc(((1 << 31) - 1) * g), oh.alloc((1 << 31) * g))
    assert hi == ((1 << 31) - 1) * g   # ends at granule 2^32 - 1
    assert gh.free(hi) == oh.free(hi) == 0
    assert np.array_equal(gh.state(), oh.state())
    assert gh.free(lo) == oh.free(lo) == 0
    assert np.array_equal(gh.state(), oh.state())
    assert gh.alloc(A) == oh.alloc(A)
    assert np.array_equal(gh.state(), oh.state())
    gh.close()


@pytest.mark.parametrize("algo", (0, 1, 2, 3, 4))
def test_partial_free_calls_match_oracle(algo):
    """hda_free_partial at random offsets (block starts, interior granule
    boundaries, unaligned, free space) against the oracle's partial free."""
    print(f"case: call-by-call partial frees algo {algo}", flush=True)
    A, g = 1 << 16, 32
    gh = hda.Heap(A, g, algo, meta_cap=512)
    oh = oracle.Heap(algo, A, g)
    rng = np.random.default_rng(40 + algo)
    live = {}
    for step in range(300):
        if live and rng.random() < 0.5:
            a = int(rng.choice(sorted(live)))
            kind = rng.integers(4)
            off = (a if kind == 0 else a + g * int(rng.integers(0, live[a] // g)) if kind == 1
                   else a + 1 if kind == 2 else int(rng.integers(0, A // g)) * g)
            r = gh.free_partial(off)
            assert r == oh.free_partial(off), (step, off)
            if r == 0:
                live = {x: s for x, s in oracle.parse_state(oh.state(), algo)["live"]}
        else:
            size = int(rng.integers(1, 3000))
            r = gh.alloc(size)
            assert r == oh.alloc(size), step
            if r >= 0:
                live = {x: s for x, s in oracle.parse_state(oh.state(), algo)["live"]}
        if step % 50 == 0:
            assert np.array_equal(gh.state(), oh.state())
    assert np.array_equal(gh.state(), oh.state())
    gh.close()


@pytest.mark.parametrize("algo", (0, 3))
def test_bad_and_double_free(algo):
    print(f"case: bad free algo {algo}", flush=True)
    gh = hda.Heap(4096, 16, algo)
    a = gh.alloc(100)
    gh.alloc(100)
    before = gh.state()
    assert gh.free(a + 16) == hda.HDA_E_BADFREE
    assert gh.free(-16) == hda.HDA_E_BADFREE
    assert gh.free(1 << 20) == hda.HDA_E_BADFREE
    assert np.array_equal(gh.state(), before)
    assert gh.free(a) == 0
    after = gh.state()
    assert gh.free(a) == hda.HDA_E_BADFREE
    assert np.array_equal(gh.state(), after)


def test_create_rejects_bad_arguments():
    for A, g, algo in ((1000, 16, 0), (1024, 24, 0), (1024, 16, 9), (0, 16, 0),
                       (1 << 40, 16, 0)):
        with pytest.raises(hda.HdaError) as e:
            hda.Heap(A, g, algo)
        assert e.value.code == hda.HDA_E_INVAL


def test_metadata_budget_admission():
    print("case: metadata budget", flush=True)
    held0 = hda.lib().hda_set_meta_budget(0)
    one = hda.Heap(1 << 20, 64, 3, meta_cap=256)
    per_heap = hda.lib().hda_set_meta_budget(0) - held0
    assert per_heap > 0
    hda.lib().hda_set_meta_budget(held0 + 2 * per_heap)
    two = hda.Heap(1 << 20, 64, 3, meta_cap=256)
    with pytest.raises(hda.HdaError) as e:
        hda.Heap(1 << 20, 64, 3, meta_cap=256)
    assert e.value.code == hda.HDA_E_NOMETA
    one.close()                                   # releases budget
    three = hda.Heap(1 << 20, 64, 3, meta_cap=256)
    assert three.alloc(1000) == 0
    hda.lib().hda_set_meta_budget(0)
    two.close()
    three.close()


def test_paper_analog_trace_matches_oracle():
    """The per-call harness the benchmark compares with hipMalloc / hipFree:
    its heap side returns the oracle's results on the stand-in trace."""
    import ctypes
    from paper_2405_07079_amd import build as hip_build
    from paper_2405_07079_amd import workloads as W
    print("case: paper-analog trace through the call-by-call harness", flush=True)
    A = ctypes.CDLL(hip_build.ANALOG)
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    A.hda_analog_heap.restype = ctypes.c_int
    A.hda_analog_heap.argtypes = [vp, i64, u64, u64, ctypes.c_int, ctypes.c_uint32, vp, vp]
    b = W.paper_analog(n=1500)
    req = np.ascontiguousarray(b.req, np.int64)
    lat, res = np.zeros(len(req), np.int64), np.zeros(len(req), np.int64)
    rc = A.hda_analog_heap(req.ctypes.data, len(req), int(b.arena[0]), int(b.align[0]),
                           int(b.algo[0]), 1024, lat.ctypes.data, res.ctypes.data)
    assert rc == 0
    exp, _ = oracle.replay_heap(int(b.algo[0]), int(b.arena[0]), int(b.align[0]), req)
    assert np.array_equal(res, exp)
    assert (lat[req >= 0] > 0).all()


# ---------------------------------------------------------------------------
# Resuming a heap from a canonical state (hda_heap_load)
# ---------------------------------------------------------------------------

def drive(gh, oh, ops):
    """Apply (kind, value) ops to a GPU heap and its oracle twin: ("a", size)
    allocates, ("f", draw) frees the oracle's live[(draw * L) >> 32]."""
    out = []
    for kind, v in ops:
        if kind == "a":
            r = gh.alloc(v)
            assert r == oh.alloc(v)
        else:
            live = oracle.parse_state(oh.state(), oh.algo)["live"]
            if not live:
                out.append(None)
                continue
            x = live[(v * len(live)) >> 32][0]
            r = gh.free(x)
            assert r == oh.free(x) == 0
        out.append(r)
    return out


def random_ops(seed, n, hi=3000):
    rng = np.random.default_rng(seed)
    return [("a", int(rng.integers(0, hi))) if rng.random() < 0.6
            else ("f", int(rng.integers(0, 1 << 32))) for _ in range(n)]


@pytest.mark.parametrize("algo", (0, 1, 2, 3, 4))
def test_load_resumes_the_heap(algo):
    """Run k calls, dump, load the dump into a fresh heap and continue: every
    result and the final state equal an uninterrupted oracle run."""
    print(f"case: heap load, algo {algo}", flush=True)
    A, g = 1 << 16, 32
    ops = random_ops(70 + algo, 500)
    oh = oracle.Heap(algo, A, g)                 # uninterrupted
    first = hda.Heap(A, g, algo, meta_cap=512)
    drive(first, oh, ops[:250])
    dumped = first.state()
    assert np.array_equal(dumped, oh.state())
    first.close()
    second = hda.Heap(A, g, algo, meta_cap=512)
    assert second.load(dumped) == hda.HDA_OK
    assert np.array_equal(second.state(), dumped)
    drive(second, oh, ops[250:])
    assert np.array_equal(second.state(), oh.state())
    second.close()


@pytest.mark.parametrize("algo", (0, 1, 2, 3, 4))
def test_load_a_replayed_state(algo):
    """A state the oracle reached by replaying a trace of the benchmark's
    shape (16 MiB, hundreds of blocks) is loaded into a GPU heap; both then
    continue with the same calls."""
    from paper_2405_07079_amd import workloads as W
    print(f"case: load a replayed state, algo {algo}", flush=True)
    b = W.uniform_batch(seed=2, heaps=1, n=6000, algo=algo)
    A, g = int(b.arena[0]), int(b.align[0])
    oh = oracle.Heap(algo, A, g)
    oh.replay(b.req)
    gh = hda.Heap(A, g, algo, meta_cap=4096)
    assert gh.load(oh.state()) == hda.HDA_OK
    drive(gh, oh, random_ops(90 + algo, 400, hi=1 << 20))
    assert np.array_equal(gh.state(), oh.state())
    gh.close()


def malformed(state, algo):
    """(name, bad state) pairs derived from a valid canonical state."""
    st = [int(x) for x in state]
    p = oracle.parse_state(st, algo)
    nf, nl = len(p["free"]), len(p["live"])
    out = [("truncated", st[:-1]), ("extra word", st + [0])]
    if nf >= 2:
        s2 = list(st)
        s2[1], s2[3] = s2[3], s2[1]                      # free blocks out of order
        out.append(("free order", s2))
    if nl >= 1:
        s2 = list(st)
        s2[2 + 2 * nf + 1] += 16                         # first live block moved: overlap
        out.append(("overlap", s2))
        s2 = list(st)
        s2[2 + 2 * nf + 2] += 1                          # unaligned size
        out.append(("unaligned", s2))
    rover_at = 2 + 2 * nf + 2 * nl
    s2 = list(st)
    s2[rover_at] = 12345 if algo == 1 else 0
    out.append(("rover", s2))
    if algo in (3, 4):
        s2 = list(st)
        s2[rover_at + 1] ^= 1 << 62                      # bitmap disagrees with the lists
        out.append(("bitmap", s2))
    return out


@pytest.mark.parametrize("algo", (0, 1, 2, 3, 4))
def test_load_rejects_malformed_states(algo):
    print(f"case: heap load of malformed states, algo {algo}", flush=True)
    A, g = 1 << 16, 32
    oh = oracle.Heap(algo, A, g)
    src = hda.Heap(A, g, algo, meta_cap=512)
    drive(src, oh, random_ops(110 + algo, 120))
    good = src.state()
    src.close()
    gh = hda.Heap(A, g, algo, meta_cap=512)
    gh.alloc(96)
    before = gh.state()
    for name, bad in malformed(good, algo):
        assert gh.load(np.array(bad, np.int64)) == hda.HDA_E_INVAL, name
        assert np.array_equal(gh.state(), before), name
    # a state of another arena, alignment or algorithm
    other = hda.Heap(A * 2, g, algo, meta_cap=512)
    assert other.load(good) == hda.HDA_E_INVAL
    other.close()
    # more blocks than the tables hold
    small = hda.Heap(A, g, algo, meta_cap=64)
    p = oracle.parse_state(good, algo)
    if max(len(p["free"]), len(p["live"])) > 64:
        assert small.load(good) == hda.HDA_E_NOMETA
    small.close()
    gh.close()


def test_library_memory_comes_from_torch():
    """The library's own device buffers are taken from torch's caching
    allocator (installed by the binding) and given back on release; the
    allocator cannot be swapped while they are held."""
    import torch
    print("case: device allocator", flush=True)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    gh = hda.Heap(1 << 20, 64, 3, meta_cap=4096)
    m1 = torch.cuda.memory_allocated()
    assert m1 - m0 >= 4096 * 20          # free table, stamps and live table
    with pytest.raises(hda.HdaError) as e:
        hda.use_hip_allocator()
    assert e.value.code == hda.HDA_E_BUSY
    assert gh.alloc(1000) == 0
    gh.close()
    assert torch.cuda.memory_allocated() == m0
