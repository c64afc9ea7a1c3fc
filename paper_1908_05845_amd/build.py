"""Builds libsmmo.so (HIP, gfx950) in the package directory.

    python -m paper_1908_05845_amd.build

Every source in csrc/ is compiled with hipcc for gfx950 and linked into one
shared library.  Flags:
  -Xclang -target-feature -Xclang -packed-fp32-ops
        no packed FP32 instructions anywhere
  -fhip-fp32-correctly-rounded-divide-sqrt
        float32 division and sqrtf are correctly rounded, which the float32
        break decision of the spring method relies on
"""

import concurrent.futures as cf
import glob
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsmmo.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def source_hash() -> str:
    """Hash of what the library is built from: every file of csrc/ and
    include/ (name and contents) and the compiler flags.  The library
    returns the value it was built with (smmo_source_hash), and the binding
    refuses a library whose value differs from that of the sources beside it."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*")) + glob.glob(os.path.join(ROOT, "include", "*")))
    for fn in files:
        if not os.path.isfile(fn):
            continue
        h.update(os.path.relpath(fn, ROOT).encode())
        with open(fn, "rb") as f:
            h.update(f.read())
    h.update(" ".join(f for f in FLAGS if not f.startswith("/")).encode())
    return h.hexdigest()[:32]


def _compile(src: str, digest: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, '-DSMMO_SOURCE_HASH="%s"' % digest, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(verbose: bool = False) -> str:
    """Compiles every csrc/*.hip and links libsmmo.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    digest = source_hash()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, digest), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-8000:]))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
