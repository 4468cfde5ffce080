"""CPU-side checks of the C-ABI library: it is built, loads, and exports every
function that include/vie.h declares (no compute calls here)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vie.h")
LIB = os.path.join(ROOT, "paper_2508_16471_amd", "libvie.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int64_t|int|void|const char)\s+\**\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ("vie_setup", "vie_solve", "vie_farfield", "hom_g2", "vie_get_current",
              "vie_set_stream", "vie_destroy", "vie_strerror", "vie_matvec"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2508_16471_amd import vie

    for n in _declared():
        assert hasattr(vie, n), n
