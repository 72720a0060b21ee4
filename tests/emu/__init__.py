"""Build and run the device replay core under the CPU lockstep wave
emulation (test infrastructure)."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2405_07079_amd", "csrc")
_lib = None


def build():
    out = os.path.join(tempfile.gettempdir(), f"hda_emu_{os.getpid()}.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                           "-I", HERE, "-I", CSRC, os.path.join(HERE, "emu_replay.cpp"),
                           "-o", out])
    return out


def lib():
    global _lib
    if _lib is None:
        # HDA_EMU_LIB: a prebuilt emulator library (the sanitizer test's build)
        L = ctypes.CDLL(os.environ.get("HDA_EMU_LIB") or build())
        vp = ctypes.c_void_p
        u32 = ctypes.c_uint32
        L.emu_replay.restype = ctypes.c_int
        L.emu_replay.argtypes = [ctypes.c_int64] + [vp] * 10 + [ctypes.c_int] + [u32] * 4 + [vp, vp]
        _lib = L
    return _lib


def replay(batch, kf=64, kl=64, cf=4096, cl=4096, shape=2, overflowed=None):
    """Replay a workloads.Batch heap by heap in the emulator.  shape selects
    the core: general with 0 = no register part, 1 = (1, 2) chunks, 2 = (4, 8)
    chunks; lean with 3 = one, 4 = four free chunks in registers (kf/kl then
    size its LDS pool: room for kf 16-byte free and kl live entries; a heap
    that outgrows it moves to the general core with no LDS part).  kf/kl are the cold entries kept in "LDS"; cf/cl the
    table capacities.  overflowed, if given, is a uint8 array of heaps that
    took the second pass."""
    H = batch.heaps
    P = lambda a: a.ctypes.data  # noqa: E731
    arena = np.ascontiguousarray(batch.arena, np.int64)
    align = np.ascontiguousarray(batch.align, np.int64)
    algo = np.ascontiguousarray(batch.algo, np.int32)
    off = np.ascontiguousarray(batch.req_off, np.int64)
    req = np.ascontiguousarray(batch.req, np.int64)
    res = np.full(req.shape, 0x7777, np.int64)
    lens = np.diff(off)
    caps = 4 + 2 * (lens + 1) + np.where(algo == 3, 64 + lens + 1,
                                         np.where(algo == 4, 2048 + lens + 1, 0))
    so = np.zeros(H + 1, np.int64)
    np.cumsum(caps, out=so[1:])
    state = np.zeros(int(so[-1]), np.int64)
    sl = np.zeros(H, np.int64)
    status = np.zeros(H, np.int32)
    syncs = np.zeros(H, np.uint64)
    rc = lib().emu_replay(H, P(arena), P(align), P(algo), P(off), P(req), P(res), P(state),
                          P(so), P(sl), P(status), int(shape), kf, kl, cf, cl, P(syncs),
                          None if overflowed is None else P(overflowed))
    # 1: a bitmask heap's node summaries disagree with its flags
    assert rc == 0, "bitmask node summaries: end runs not exact or the longest-run bound below the true run" if rc == 1 else rc
    states = [state[so[h]:so[h] + sl[h]].copy() for h in range(H)]
    return res, states, status, syncs
