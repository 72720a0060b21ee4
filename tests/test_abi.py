"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/hda.h declares (no compute calls here)."""
import ctypes
import os
import re

from paper_2405_07079_amd import hda

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "hda.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hda_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("hda_heap_create", "hda_alloc", "hda_free", "hda_heap_destroy",
              "hda_replay", "hda_heap_state"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(hda.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_knows_every_symbol():
    assert sorted(hda.EXPORTS) == declared()


def test_strerror_without_gpu():
    assert hda.strerror(hda.HDA_E_BADFREE).startswith("free of an offset")
    assert hda.strerror(12345) == "unknown error"


def test_header_compiles_as_c_and_cpp():
    """include/hda.h stands alone for C and C++ callers."""
    import subprocess
    hdr = os.path.join(ROOT, "include", "hda.h")
    for lang, cc in (("c", "gcc"), ("c++", "g++")):
        subprocess.check_call([cc, "-fsyntax-only", "-Wall", "-Werror", "-x", lang, hdr])


def test_device_allocator_needs_both_callbacks():
    """Exactly one callback is an invalid argument (no GPU call is made)."""
    L = hda.lib()
    rc = L.hda_set_device_allocator(hda._TORCH_ALLOCATOR[0], hda.DEV_FREE(), None)
    assert rc == hda.HDA_E_INVAL
    rc = L.hda_set_device_allocator(hda.DEV_ALLOC(), hda._TORCH_ALLOCATOR[1], None)
    assert rc == hda.HDA_E_INVAL
