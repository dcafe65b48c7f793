"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2607_15413_amd import fsz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "fsz.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsz_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fsz.load_library()
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert set(declared) == set(fsz.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_bound_matches_format_arithmetic():
    def ref(n):
        nb = -(-n // 32)
        nt = -(-n // 256)
        return 32 + (nb + 15) // 16 * 16 + 4 * nt + 128 * nb
    for n in (0, 1, 31, 32, 33, 255, 256, 257, 1 << 20, 25_000_000, 1 << 27, (1 << 33) + 5):
        assert fsz.fsz_compressed_bound(n) == ref(n)


def test_status_strings():
    for s in range(9):
        assert isinstance(fsz.fsz_status_string(s), str)
    assert fsz.fsz_status_string(0) == "ok"


def test_invalid_arguments_rejected_on_host():
    # argument checks happen before any device work, so they run without a GPU
    st, _ = fsz.fsz_compress(0, 10, 0, 1e-3, 0, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 10, 5, 1e-3, 16, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 10, 1, float("nan"), 16, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 10, 1, -1.0, 16, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(18, 10, 1, 1e-3, 16, 1000, None)  # misaligned input
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 1000, 1, 1e-3, 16, 40, None)  # below the rate header size
    assert st == fsz.FSZ_ERR_CAPACITY
    assert fsz.fsz_decompress(16, 8, 16, 10, None) == fsz.FSZ_ERR_CORRUPT
    assert fsz.fsz_decompress(0, 100, 16, 10, None) == fsz.FSZ_ERR_INVALID_ARG
