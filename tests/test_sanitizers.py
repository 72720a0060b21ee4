"""The device cores (under the CPU wave emulation) and the oracle built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only, g++), then
replayed on small batches of every algorithm and core in a child process:
an out-of-bounds table access, a use after free or undefined arithmetic
aborts the child.  The sanitized builds' results must still equal each
other."""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2405_07079_amd", "csrc")
FLAGS = ["-O1", "-g", "-std=c++17", "-shared", "-fPIC", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

CHILD = r"""
import numpy as np
import emu, oracle
from paper_2405_07079_amd import workloads as W

def same(b, shape, **kw):
    res, states, status, _ = emu.replay(b, shape=shape, **kw)
    ores, ostates, _ = oracle.replay_batch(b, threads=2)
    assert (status == 0).all(), (shape, status)
    assert np.array_equal(res, ores), shape
    for h in range(b.heaps):
        assert np.array_equal(states[h], ostates[h]), (shape, h)

parts = [W.uniform_batch(seed=40 + a, heaps=1, n=400, algo=a) for a in range(5)]
parts += [W.random_tiny(7 + a, 200, 200, align=16, algo=a, max_granules=40, p_partial=0.3)
          for a in range(5)]
b = W.concat(parts)
same(b, 1, kf=64, kl=64, cf=512, cl=512)
same(b, 3, kf=64, kl=64, cf=512, cl=512)
same(b, 6, kf=64, kl=64, cf=512, cl=512)
tiny = W.uniform_batch(seed=7, heaps=1, arena=1 << 24, align=16, n=1500, p_alloc=0.6,
                       lo=16, hi=160, algo=W.NEXT_FIT)
same(tiny, 6, kf=64, kl=64, cf=4096, cl=8192)
bm = W.concat([W.uniform_batch(seed=50, heaps=1, n=300, algo=W.BITMAP),
               W.random_tiny(9, 300, 200, align=16, algo=W.BITMAP, max_granules=40)])
same(bm, 5, cf=1024, cl=1024)
edge = W.max_arena_batch()
same(edge, 3, kf=64, kl=64, cf=64, cl=64)
same(edge, 6, kf=64, kl=64, cf=64, cl=192)
print("sanitized replays ok")
"""


def runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_cores_and_oracle_under_asan_and_ubsan():
    asan = runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for g++ here")
    with tempfile.TemporaryDirectory() as d:
        emu_so = os.path.join(d, "emu_asan.so")
        orc_so = os.path.join(d, "oracle_asan.so")
        subprocess.check_call(["g++", *FLAGS, "-I", os.path.join(HERE, "emu"), "-I", CSRC,
                               os.path.join(HERE, "emu", "emu_replay.cpp"), "-o", emu_so])
        subprocess.check_call(["g++", *FLAGS, "-pthread",
                               os.path.join(ROOT, "oracle", "hda_oracle.cpp"), "-o", orc_so])
        env = dict(os.environ, LD_PRELOAD=asan, HDA_EMU_LIB=emu_so, HDA_ORACLE_LIB=orc_so,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
                   PYTHONPATH=os.pathsep.join([ROOT, HERE]))
        p = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True,
                           text=True, timeout=1200)
        tail = (p.stdout + p.stderr)[-4000:]
        assert p.returncode == 0, tail
        assert "sanitized replays ok" in p.stdout
        assert "ERROR: AddressSanitizer" not in p.stderr, tail
        assert "runtime error" not in p.stderr, tail
