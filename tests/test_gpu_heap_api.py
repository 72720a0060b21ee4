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
