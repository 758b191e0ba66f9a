"""The C-ABI library loads, exports every entry point include/hx.h declares,
and behaves on a host-only context (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1810_11482_amd as hx

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:hx_status|const char\*)\s+(hx_\w+)\s*\(", text,
                                 flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 25
    lib = ctypes.CDLL(hx.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    assert hx.hx_status_string(0) == "HX_OK"
    assert hx.hx_status_string(hx.HX_ERR_DEP_FAILED) == "HX_ERR_DEP_FAILED"
    assert hx.hx_status_string(hx.HX_PENDING) == "HX_PENDING"
    assert hx.hx_status_string(-99) == "HX_UNKNOWN_STATUS"


def test_null_and_bad_arguments():
    assert hx.lib.hx_device_count(None) == hx.HX_ERR_ARG
    assert hx.lib.hx_ctx_create(-1, None, None) == hx.HX_ERR_ARG
    assert hx.lib.hx_ctx_destroy(None) == hx.HX_ERR_INVALID
    assert hx.lib.hx_wait(None, 5, 0) == hx.HX_ERR_INVALID
