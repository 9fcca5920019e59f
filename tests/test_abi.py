"""The C-ABI library loads and exports every entry point include/vbdr.h
declares; host-side argument checks that need no GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vbdr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vbdr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def V():
    from paper_1810_13132_amd import vbdr
    return vbdr


def test_header_lists_the_boundary():
    names = declared_functions()
    for n in ("vbdr_sketch_create", "vbdr_scan_slice", "vbdr_advance_slice", "vbdr_estimate"):
        assert n in names


def test_library_exports_every_declared_symbol(V):
    lib = V.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(V.EXPORTS) == sorted(declared_functions())


@pytest.mark.parametrize("m,g,k,layout,why", [
    (1000, 3, 4, 0, "g not a power of two"),
    (1000, 1, 4, 0, "g below 2"),
    (1 << 20, 1 << 17, 4, 0, "g above 65536"),
    (256, 256, 4, 0, "m not above g"),
    (1 << 32, 256, 4, 0, "m not below 2^32"),
    (1000, 16, 0, 0, "k = 0"),
    (1000, 16, 255, 0, "k above 254"),
    (1000, 16, 4, 7, "unknown layout"),
])
def test_create_rejects_bad_parameters(V, m, g, k, layout, why):
    lib = V.lib()
    h = C.c_void_p()
    rc = lib.vbdr_sketch_create_layout(m, g, k, 0, layout, C.byref(h))
    assert rc == -1, why
    assert not h.value
    assert lib.vbdr_last_error().decode()


def test_null_handles_rejected(V):
    lib = V.lib()
    assert lib.vbdr_scan_slice(None, None, 5, None) == -1
    assert lib.vbdr_advance_slice(None, None) == -1
    assert lib.vbdr_estimate(None, None, 3, None, None) == -1
    assert lib.vbdr_sketch_create(1000, 16, 4, 0, None) == -1
    lib.vbdr_sketch_destroy(None)  # no-op
    info = V.Info()
    assert lib.vbdr_sketch_info(None, C.byref(info)) == -1
