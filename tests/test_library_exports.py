"""The built C-ABI library loads and exports every symbol include/xeng.h declares (no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "xeng.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(xeng_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["xeng_create", "xeng_correlate", "xeng_dump", "xeng_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1411_3751_amd import xeng
    if not os.path.exists(xeng.LIB_PATH):
        pytest.skip("libxeng.so not built")
    lib = xeng.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(xeng.EXPORTS)


def test_strerror_without_device():
    from paper_1411_3751_amd import xeng
    if not os.path.exists(xeng.LIB_PATH):
        pytest.skip("libxeng.so not built")
    lib = xeng.load()
    assert lib.xeng_strerror(2) == b"exactness bound exceeded"
    assert lib.xeng_strerror(0) == b"ok"
