"""The C-ABI library loads on the CPU and exports every symbol the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsvdmi.h")
LIB = os.path.join(ROOT, "paper_1902_03070_amd", "libtsvdmi.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_header_lists_the_boundary_calls():
    names = declared_functions()
    for want in ("tsvd_dct", "tsvt_dct", "tprod_dct", "complete_tensor", "tsvt_dct_batched",
                 "tsvd_server_create", "tsvd_server_submit", "tsvd_server_poll"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_match_header():
    from paper_1902_03070_amd import _lib

    assert sorted(_lib.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_context_is_rejected_without_gpu():
    from paper_1902_03070_amd import _lib

    assert _lib.lib.tsvt_dct(None, 0, 4, 4, 4, None, None, 1.0, None, None) == _lib.EINVAL
    assert _lib.lib.tsvd_set_option(None, 0, 5.0) == _lib.EINVAL
    assert _lib.lib.tsvd_last_error(None) == b"null context"
