import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # build the libraries when nothing is built (a fresh checkout), and the
    # HIP library also when it was built from other sources than the tree's
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        from oracle import build as ob
        ob.build()
    from paper_1710_08774_amd import build as hb
    lib = os.path.join(ROOT, "paper_1710_08774_amd", "libhfav.so")
    if not os.path.exists(lib) or hb.built_id(lib) != hb.source_hash():
        hb.build()
