"""Build libfnlh.so in-tree for gfx950 (hipcc cross-compiles; no GPU needed).  Each
source compiles to an object of its own, in parallel, then one link."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libfnlh.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "nn.hip", "krylov.hip", "noalloc.hip", "api.cpp", "nn.cpp", "rk.cpp", "krylov.cpp",
           "layout.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # never emit packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, err


def build(verbose: bool = True) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(OBJDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = sources()
    objs = [os.path.join(OBJDIR, os.path.basename(f) + ".o") for f in srcs]
    cmds = [[hipcc, *HIPCC_FLAGS, "-c", f, "-o", o] for f, o in zip(srcs, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, err), f in zip(results, srcs):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(f)}:\n" + err)
    tmp = LIB + ".tmp"
    # -z defs: a symbol left undefined fails the link here, not the first load on a GPU
    link = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-Wl,-z,defs", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
