"""The C ABI: liblabs.so loads on a CPU-only host and exports every entry point include/labs.h
declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "labs.h")
LIB = os.path.join(ROOT, "paper_2011_00068_amd", "liblabs.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(labs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("labs_isl", "labs_merit", "labs_walk_batch", "labs_search_submit", "labs_search_poll"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert missing == []


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_binding_lists_every_declared_symbol():
    import paper_2011_00068_amd as labs

    assert sorted(labs.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_strerror_without_device():
    lib = ctypes.CDLL(LIB)
    lib.labs_strerror.restype = ctypes.c_char_p
    assert lib.labs_strerror(0) == b"ok"
    assert lib.labs_strerror(-2) == b"sequence is not skew-symmetric"
