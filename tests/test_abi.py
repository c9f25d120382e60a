"""The C ABI library loads and exports every function include/*.h declares
(no compute calls)."""
import ctypes
import glob
import os
import re

from paper_1710_08774_amd import hfav as H

INC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions():
    names = set()
    for path in glob.glob(os.path.join(INC, "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(hfav_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "hfav_chain_create" in names and "hfav_plan" in names and "hfav_execute" in names
    lib = ctypes.CDLL(H.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string():
    assert "gfx950" in H.version()


def test_static_workspace_size_matches_header():
    text = open(os.path.join(INC, "hfav.h")).read()
    m = re.search(r"#define HFAV_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "HFAV_STATIC_WORKSPACE_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == H.STATIC_WORKSPACE_BYTES


def test_noalloc_refuses_before_touching_a_device():
    """The size and plan checks of hfav_execute_noalloc run on the host
    before any device call (the pointers below are never dereferenced)."""
    c = H.Chain(H.hdiff_spec())
    assert c.execute_noalloc_status([1], [2]) == H.ENOPLAN
    info = c.plan((512, 512, 12), mode=H.MODE_UNFUSED)
    assert info.workspace_bytes > H.STATIC_WORKSPACE_BYTES
    assert c.execute_noalloc_status([1], [2]) == H.ESIZE
    assert "static workspace" in H.last_error()


def test_bound_execute_refuses_after_a_replan():
    """Chain.bind checks the buffers once; after the chain is planned again
    the binding is stale and refuses before any device call."""
    c = H.Chain(H.hdiff_spec())
    c.plan((64, 32, 2))
    b = c.bind([0x100000], [0x900000])
    assert not b.stale()
    c.plan((64, 32, 4))
    assert b.stale()
    try:
        b(stream=0)
    except H.HfavError as e:
        assert e.code == H.ENOPLAN
    else:
        raise AssertionError("a stale binding ran")
