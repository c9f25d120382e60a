"""Build libhfav.so (host planner + gfx950 kernels) in place with hipcc.

The library carries a hash of the sources it was built from (hfav_build_id):
the binding refuses a library whose hash differs from the tree's sources, so
a source change without a rebuild cannot run old code silently."""
import hashlib
import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhfav.so")
ARCH = os.environ.get("HFAV_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def source_hash():
    """16 hex digits over the kernel and planner sources, the public headers,
    the target and the compile flags."""
    inc = os.path.join(HERE, "..", "include")
    h = hashlib.sha256()
    h.update(" ".join([ARCH] + COMMON[:-1] + DEVICE).encode())
    for d, names in ((CSRC, sorted(os.listdir(CSRC))), (inc, sorted(os.listdir(inc)))):
        for f in names:
            if not f.endswith((".cpp", ".hip", ".h")):
                continue
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def built_id(path=LIB):
    """Build id recorded in a built library (read from the file, without
    loading it), or None."""
    try:
        with open(path, "rb") as fh:
            data = fh.read()
    except OSError:
        return None
    k = data.find(b"hfav-build-id:")
    return data[k + 14:k + 30].decode("ascii", "replace") if k >= 0 else None


def _compile(src, build_id):
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC] + COMMON + ['-DHFAV_BUILD_ID="%s"' % build_id]
    if src.endswith(".hip"):
        cmd += ["-x", "hip"] + DEVICE
    else:
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False, jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    t0 = time.time()
    build_id = source_hash()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_id), sources()))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
