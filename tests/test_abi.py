"""CPU checks of the C-ABI library: it loads and exports every function that
include/tersoff.h declares; the binding declares the same set.  No compute
call is made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tersoff.h")
LIB = os.path.join(ROOT, "paper_1710_00882_amd", "libtersoff.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tersoff_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_functions():
    names = declared_functions()
    assert "tersoff_create" in names and "tersoff_compute" in names
    assert len(names) >= 10


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libtersoff.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_exports_are_c_symbols():
    if not os.path.exists(LIB):
        pytest.skip("libtersoff.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tersoff_[a-z_0-9]+)\b", out))
    assert set(declared_functions()) <= exported


def test_binding_matches_header():
    from paper_1710_00882_amd import _lib
    assert set(_lib.SYMBOLS) == set(declared_functions())


def test_strerror_without_device(lib):
    lib.tersoff_strerror.restype = ctypes.c_char_p
    assert lib.tersoff_strerror(0) == b"ok"
    assert b"box" in lib.tersoff_strerror(-3)


def test_create_rejects_bad_arguments_without_device(lib):
    # argument validation happens before any device call
    import numpy as np
    from paper_1710_00882_amd import workloads as W
    h = ctypes.c_void_p()
    lib.tersoff_create.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
    tab = np.ascontiguousarray(W.si_table())
    assert lib.tersoff_create(tab.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(h)) == -1
    assert lib.tersoff_create(tab.ctypes.data_as(ctypes.c_void_p), 5, ctypes.byref(h)) == -1
    bad = tab.copy(); bad[0, 0, 0, 6] = -1.0      # eta <= 0
    assert lib.tersoff_create(bad.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(h)) == -1
    bad = tab.copy(); bad[0, 0, 0, 13] = 2.0      # m not in {1, 3}
    assert lib.tersoff_create(bad.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(h)) == -1


def test_missing_library_raises(tmp_path, monkeypatch):
    from paper_1710_00882_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
