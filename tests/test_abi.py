"""The C-ABI library loads and exports every function the public header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmsvd.h")
LIB = os.path.join(ROOT, "paper_2601_11626_amd", "libcmsvd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmsvd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for f in ("cmsvd_update", "cmsvd_merge_errors", "cmsvd_cluster", "cmsvd_create", "cmsvd_destroy",
              "cmsvd_last_error"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcmsvd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for f in declared_functions():
        assert hasattr(lib, f), f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcmsvd.so not built")
def test_binding_lists_the_exports():
    import paper_2601_11626_amd as cm

    assert sorted(cm.EXPORTS) == declared_functions()
