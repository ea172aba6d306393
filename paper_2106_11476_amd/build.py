"""Build libfw2.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to an object of its own in parallel (the kernel sources
dominate the build time), then one hipcc line links the shared library.
"""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfw2.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("kernels.hip", "step_p2.hip", "step_v2.hip", "step_p3.hip", "step_v3.hip", "batch.hip",
                     "adjoint.hip", "halo.hip", "fw2.cpp", "setup.cpp")]
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         # no packed FP32 instructions in any device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=True, jobs=None):
    """Compile every source into paper_2106_11476_amd/libfw2.so (always rebuilds)."""
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    with tempfile.TemporaryDirectory(prefix="fw2_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]

        def compile_one(k):
            cmd = [cc] + FLAGS + inc + ["-c", SOURCES[k], "-o", objs[k]]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        n = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=n) as ex:
            list(ex.map(compile_one, range(len(SOURCES))))
        tmp = LIB + ".tmp"
        cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
