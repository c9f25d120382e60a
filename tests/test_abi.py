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
