"""CPU checks of the C ABI boundary: the built library loads and exports every
function include/rsi.h declares, the binding's host logic, and the loud
failure when the library is missing.  No device call is made here."""
import ctypes
import os
import re

import pytest

from paper_2209_02878_amd import rsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsi_[a-z_]+)\s*\(", src)))


def _lib_or_skip():
    if not os.path.exists(rsi.LIB_PATH):
        pytest.skip("librsi.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(rsi.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rsi_build", "rsi_rebuild", "rsi_refit", "rsi_query", "rsi_destroy",
                 "rsi_spill_info", "rsi_spill_read", "rsi_status_str", "rsi_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(rsi.EXPORTED) == _declared()


def test_status_strings_without_device():
    L = _lib_or_skip()
    L.rsi_status_str.restype = ctypes.c_char_p
    assert L.rsi_status_str(0) == b"ok"
    assert L.rsi_status_str(1) == b"invalid argument"


def test_null_handle_is_rejected_without_device():
    L = _lib_or_skip()
    L.rsi_refit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    assert L.rsi_refit(None, None, 0, None) == rsi.RSI_E_INVALID
    L.rsi_last_error.restype = ctypes.c_char_p
    assert b"NULL handle" in L.rsi_last_error()
    out = ctypes.c_void_p()
    L.rsi_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    assert L.rsi_build(None, -1, None, 0, None, None, ctypes.byref(out)) == rsi.RSI_E_INVALID
    assert L.rsi_build(None, 0, None, 5, None, None, ctypes.byref(out)) == rsi.RSI_E_INVALID


def test_parse_mode():
    assert rsi.parse_mode("bool") == 1
    assert rsi.parse_mode("first|all") == 6
    assert rsi.parse_mode("bool+first+all") == 7
    assert rsi.parse_mode(4) == 4


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(rsi, "_lib", None)
    monkeypatch.setattr(rsi, "LIB_PATH", os.path.join(ROOT, "does-not-exist", "librsi.so"))
    with pytest.raises(RuntimeError, match="not built"):
        rsi.lib()
