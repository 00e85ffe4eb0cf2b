"""The C-ABI library loads and exports every function declared in include/gp.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1502_07451_amd", "libgp.so")


def declared_functions():
    names = set()
    with open(os.path.join(ROOT, "include", "gp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    for m in re.finditer(r"\b(gp_\w+)\s*\(", text):
        names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("gp_create", "gp_partition", "gp_destroy", "gp_ratio_from_times",
                 "gp_strerror", "gp_options_default"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgp.so not built")
def test_host_only_entry_points():
    # these touch no device
    lib = ctypes.CDLL(LIB)
    lib.gp_ratio_from_times.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    out = (ctypes.c_int64 * 2)()
    assert lib.gp_ratio_from_times(400, 100, out) == 0 and list(out) == [1, 4]
    assert lib.gp_ratio_from_times(0, 0, out) == 1
    lib.gp_strerror.restype = ctypes.c_char_p
    assert b"self loop" in lib.gp_strerror(4)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgp.so not built")
def test_model_load_rejects_bad_files(tmp_path):
    # both checks happen before the library touches the device
    lib = ctypes.CDLL(LIB)
    lib.gp_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p(1)
    assert lib.gp_model_load(os.fsencode(str(tmp_path / "missing.bin")), ctypes.byref(h)) == 1
    assert not h.value
    short = tmp_path / "short.bin"
    short.write_bytes(b"\0" * (2 * 25153 - 2))
    assert lib.gp_model_load(os.fsencode(str(short)), ctypes.byref(h)) == 9
    long_ = tmp_path / "long.bin"
    long_.write_bytes(b"\0" * (2 * 25153 + 2))
    assert lib.gp_model_load(os.fsencode(str(long_)), ctypes.byref(h)) == 9
    assert not h.value
