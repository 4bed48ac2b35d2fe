"""Build libepw.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1604_03525_amd.build

Every call recompiles every translation unit (object files go to
paper_1604_03525_amd/_build/) and links paper_1604_03525_amd/libepw.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libepw.so")
ARCH = os.environ.get("EPW_OFFLOAD_ARCH", "gfx950")

SOURCES = ["errors.cpp", "host_lattice.cpp", "timing.cpp", "api.cpp", "k_eigh.hip", "k_vertex.hip",
           "k_gemm.hip", "k_backward.hip", "k_spectral.hip", "k_polar.hip", "k_transport.hip",
           "k_check.hip", "noalloc.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed fp32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    return src, obj, res.returncode, out


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    failed = False
    for src, _, rc, out in results:
        if out.strip() and (verbose or rc != 0):
            print("[%s]\n%s" % (src, out), file=sys.stderr)
        failed |= rc != 0
    if failed:
        raise RuntimeError("libepw: compilation failed")
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + \
        [obj for _, obj, _, _ in results]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("libepw: link failed\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
