"""The C-ABI boundary without a GPU: the built library loads, exports every
function that include/zoomhash.h declares, and the ctypes binding declares
the same set of functions. No call that needs a device is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zoomhash.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(zh_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1004_3980_amd import build
    path = os.path.join(ROOT, "paper_1004_3980_amd", "libzoomhash.so")
    if not os.path.exists(path):
        build.build()
    return ctypes.CDLL(path)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("zh_build_tables", "zh_query", "zh_lle_weights", "zh_reconstruct", "zh_backproject",
                     "zh_backward", "zh_create", "zh_destroy", "zh_last_error"):
        assert required in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1004_3980_amd import zoomhash
    bound = set(zoomhash.SIGNATURES) | {"zh_last_error"}
    assert set(declared_functions()) <= bound, sorted(set(declared_functions()) - bound)
