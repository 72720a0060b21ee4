"""CPU oracle for allocator replay -- TEST INFRASTRUCTURE ONLY.

Loads ``libhda_oracle.so`` (built from ``hda_oracle.cpp`` by :func:`build`)
through ctypes.  Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hda_oracle.cpp")
LIB = os.path.join(HERE, "libhda_oracle.so")

FIRST_FIT, NEXT_FIT, BEST_FIT, SEG_FIT, TLSF, BITMAP = 0, 1, 2, 3, 4, 5


def n_lists(algo: int) -> int:
    """Class lists in a state dump: 64 (segregated fit), 64 * 32 (TLSF), 0."""
    return 64 if algo == SEG_FIT else 64 * 32 if algo == TLSF else 0
E_INVAL, E_BADFREE = -2, -3

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (no GPU code involved)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("HDA_ORACLE_LIB")   # a planted-mistake build (tests)
        if path is None:
            path = LIB
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
        L = ctypes.CDLL(path)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.orc_heap_new.restype = vp
        L.orc_heap_new.argtypes = [i32, i64, i64]
        L.orc_heap_delete.argtypes = [vp]
        L.orc_alloc.restype = i64
        L.orc_alloc.argtypes = [vp, i64]
        L.orc_dealloc.restype = i32
        L.orc_dealloc.argtypes = [vp, i64]
        L.orc_dealloc_partial.restype = i32
        L.orc_dealloc_partial.argtypes = [vp, i64]
        L.orc_dump.restype = i64
        L.orc_dump.argtypes = [vp, vp, i64]
        L.orc_stats.argtypes = [vp, vp]
        L.orc_replay_on.argtypes = [vp, i64, vp, vp]
        L.orc_replay_batch.restype = i32
        L.orc_replay_batch.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                       vp, i32]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Heap:
    """One oracle heap driven call by call."""

    def __init__(self, algo: int, arena: int, align: int):
        self._h = lib().orc_heap_new(int(algo), int(arena), int(align))
        if not self._h:
            raise ValueError("invalid heap parameters")
        self.algo, self.arena, self.align = int(algo), int(arena), int(align)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_heap_delete(self._h)
            self._h = None

    def alloc(self, size: int) -> int:
        return int(lib().orc_alloc(self._h, int(size)))

    def free(self, offset: int) -> int:
        return int(lib().orc_dealloc(self._h, int(offset)))

    def free_partial(self, offset: int) -> int:
        """Free from `offset` to the end of the live block holding it (the
        whole block if `offset` is its start; sequential fits only)."""
        return int(lib().orc_dealloc_partial(self._h, int(offset)))

    def replay(self, req) -> np.ndarray:
        req = np.ascontiguousarray(req, dtype=np.int64)
        res = np.empty_like(req)
        lib().orc_replay_on(self._h, req.shape[0], _ptr(req), _ptr(res))
        return res

    def state(self) -> np.ndarray:
        n = lib().orc_dump(self._h, None, 0)
        buf = np.empty(n, np.int64)
        lib().orc_dump(self._h, _ptr(buf), n)
        return buf

    def stats(self):
        out = np.zeros(2, np.uint64)
        lib().orc_stats(self._h, _ptr(out))
        return int(out[0]), int(out[1])


def replay_heap(algo, arena, align, req):
    """Replay one heap from its initial state: (results, state)."""
    h = Heap(algo, arena, align)
    res = h.replay(req)
    return res, h.state()


def state_capacity(algo: int, n_requests: int, cap_blocks: int | None = None):
    """Words needed for a state dump when at most ``cap_blocks`` blocks exist."""
    b = n_requests + 1 if cap_blocks is None else cap_blocks
    return 4 + 4 * b + (n_lists(algo) + b if n_lists(algo) else 0)


def replay_batch(batch, threads: int = 1, want_state: bool = True,
                 want_stats: bool = False, state_blocks: int | None = None):
    """Replay every heap of a ``workloads.Batch``.

    Returns ``(res, states, stats)``: results aligned with ``batch.req``, a list
    of per-heap state arrays (or None) and per-heap (examined, touched) counts
    (or None).  ``state_blocks`` bounds the blocks a heap's state slot is sized
    for (default: one more than its requests); a heap whose state needs more
    words gets an empty array, which no real state equals.
    """
    H = batch.heaps
    arena = np.ascontiguousarray(batch.arena, np.int64)
    align = np.ascontiguousarray(batch.align, np.int64)
    algo = np.ascontiguousarray(batch.algo, np.int32)
    off = np.ascontiguousarray(batch.req_off, np.int64)
    req = np.ascontiguousarray(batch.req, np.int64)
    res = np.empty_like(req)
    state = state_off = state_len = None
    if want_state:
        lens = np.diff(off)
        caps = np.array([state_capacity(int(a), int(n),
                                        None if state_blocks is None
                                        else min(int(n) + 1, int(state_blocks)))
                         for a, n in zip(algo, lens)], np.int64)
        state_off = np.zeros(H + 1, np.int64)
        np.cumsum(caps, out=state_off[1:])
        state = np.empty(int(state_off[-1]), np.int64)
        state_len = np.zeros(H, np.int64)
    stats = np.zeros(2 * H, np.uint64) if want_stats else None
    rc = lib().orc_replay_batch(H, _ptr(arena), _ptr(align), _ptr(algo), _ptr(off),
                                _ptr(req), _ptr(res), _ptr(state), _ptr(state_off),
                                _ptr(state_len), _ptr(stats), int(threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the batch (code {rc})")
    states = None
    if want_state:
        states = [state[state_off[i]:state_off[i] + state_len[i]].copy()
                  if state_len[i] <= state_off[i + 1] - state_off[i] else np.zeros(0, np.int64)
                  for i in range(H)]
    return res, states, (stats.reshape(H, 2) if want_stats else None)


def parse_state(st, algo: int):
    """Split a canonical state dump into a dict."""
    st = [int(x) for x in st]
    p = 0
    nf = st[p]; p += 1
    free = [(st[p + 2 * i], st[p + 2 * i + 1]) for i in range(nf)]; p += 2 * nf
    nl = st[p]; p += 1
    live = [(st[p + 2 * i], st[p + 2 * i + 1]) for i in range(nl)]; p += 2 * nl
    rover = st[p]; bitmap = st[p + 1] & ((1 << 64) - 1); p += 2
    lists = None
    if n_lists(algo):
        lists = []
        for _ in range(n_lists(algo)):
            n = st[p]; p += 1
            lists.append(st[p:p + n]); p += n
    assert p == len(st), "malformed state"
    return dict(free=free, live=live, rover=rover, bitmap=bitmap, lists=lists)
