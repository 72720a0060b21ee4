"""Build the gfx950 shared library ``libhda.so`` in-tree with hipcc."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhda.so")
SOURCES = ["hda_replay.hip", "hda_heap.hip", "hda_serve.hip", "hda_bitmap.hip"]
HEADERS = ["hda_wave.h", "hda_core.h", "hda_lean.h", "hda_ordered.h", "hda_bitmap.h", "hda_replay_body.h",
           "hda_heap_dev.h", "hda_mem.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         # packed FP32 instructions stay off in every device compile
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # branches on wave-uniform values stay plain scalar branches: the
         # cores branch only on uniform values, and structurizing those
         # regions as if they could diverge made the request loops copy
         # the heap's registers on every request
         "-mllvm", "-structurizecfg-skip-uniform-regions=true",
         "-Wall", "-Wno-unused-function"]


# the per-call latency harness of the benchmark's vendor comparison: host
# code only, linked against libhda.so
ANALOG = os.path.join(PKG, "libhda_analog.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs,
           "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    tmp = ANALOG + f".tmp{os.getpid()}"
    cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "hda_analog.cpp"),
           "-L", PKG, "-lhda", "-Wl,-rpath,$ORIGIN", "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, ANALOG)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
