"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "osam.h")
LIB = os.path.join(ROOT, "paper_2511_20687_amd", "libosam.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ("create_subdomain", "learn_opinf", "schwarz_step", "run"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosam.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosam.so not built")
def test_binding_declares_the_same_symbols():
    from paper_2511_20687_amd import osam
    assert sorted(osam.EXPORTED) == _declared()
    lib = osam.load_library()
    assert lib.osam_version() >= 10000
