"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dhtrace.h")
LIB = os.path.join(ROOT, "paper_1603_05988_amd", "libdhtrace.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dht_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdhtrace.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_1603_05988_amd import _lib
    assert set(declared_symbols()) == set(_lib.SIGNATURES)


def test_version_and_error_strings(lib):
    lib.dht_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.dht_version()
    lib.dht_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.dht_last_error(), bytes)
