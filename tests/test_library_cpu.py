"""Host-side checks of libcg that need no GPU: the library loads, exports
every entry point include/cg.h declares, sizes scratch, and rejects bad
arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2207_04350_amd import cg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cg.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(cg_\w+)\(", text, re.M)))


def test_header_declares_the_five_steps():
    names = _declared()
    for step in ("cg_mask_branches", "cg_components", "cg_partition", "cg_induce", "cg_assemble"):
        assert step in names


def test_library_exports_every_declared_symbol():
    lib = cg.lib()
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_footprint_grows_with_the_graph():
    a = cg.footprint(1000, 2000, 8)
    b = cg.footprint(100000, 200000, 8)
    c = cg.footprint(100000, 200000, 4096)
    assert 0 < a < b < c
    s1 = cg.sizes(1000, 2000, 5000, 8)
    s2 = cg.sizes(1000, 2000, 6000, 8)
    s3 = cg.sizes(1000, 2000, 6000, 8, coords=True)
    assert s2["graph"] - s1["graph"] == 4000 and s2["outputs"] - s1["outputs"] == 4000
    assert s3["graph"] - s2["graph"] == 8 * 2000 and s3["outputs"] == s2["outputs"]
    assert s1["scratch"] == a
    for bad in ((-1, 0, 0, 8), (10, -1, 0, 8), (10, 10, 0, 0), (10, 10, 0, 70000),
                (10, 10, 1 << 62, 8)):
        with pytest.raises(cg.CgError):
            cg.sizes(*bad)


def test_null_arguments_rejected_on_host():
    lib = cg.lib()
    g = cg.CgGraph()
    g.n, g.m = 10, 0
    assert lib.cg_mask_branches(None, ctypes.byref(g), None, None, None) == cg.CG_EINVAL
    assert b"NULL" in lib.cg_last_error() or lib.cg_last_error()
    assert lib.cg_partition(None, ctypes.byref(g), None, None, 0, 2, 0, None, None) == cg.CG_EINVAL
    assert lib.cg_partition(None, ctypes.byref(g), None, None, 70000, 2, 0, None, None) == cg.CG_EINVAL
    # an unknown weight, and pre without post, are argument errors
    assert lib.cg_partition(None, ctypes.byref(g), None, None, 4, 2, 7, None, None) == cg.CG_EINVAL
    pre = (ctypes.c_uint32 * 1)()
    g.row_ptr = ctypes.cast(pre, ctypes.c_void_p)   # checked on the host only, never read
    g.pre = ctypes.cast(pre, ctypes.c_void_p)
    assert lib.cg_mask_branches(None, ctypes.byref(g), None, None, None) == cg.CG_EINVAL
    assert b"pre and post" in lib.cg_last_error()
    g.pre = g.row_ptr = None
    g.n = 1 << 30
    assert lib.cg_components(None, ctypes.byref(g), None, None, None) == cg.CG_EINVAL


def test_reduce_arguments_checked_on_host():
    lib = cg.lib()
    g = cg.CgGraph()
    g.n, g.m = 4, 0
    buf = (ctypes.c_int32 * 8)()
    g.row_ptr = ctypes.cast(buf, ctypes.c_void_p)   # checked on the host only, never read
    # no outputs, no context: argument errors before any device work
    assert lib.cg_reduce(None, ctypes.byref(g), 0, None, None, None, None, None, None, None,
                         None) == cg.CG_EINVAL
    assert b"NULL" in lib.cg_last_error()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.cg_reduce(None, ctypes.byref(g), 0, p, p, p, p, p, p, p, None) == cg.CG_EINVAL
