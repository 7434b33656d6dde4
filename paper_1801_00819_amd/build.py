"""Build libbrrlsm.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbrrlsm.so")
SOURCES = ["stencil2d.hip", "march2d.hip", "march2t.hip", "stencil3d.hip",
           "march2s.hip", "bg64.hip",
           "blas.hip", "engine.hip", "ssf.hip", "ssf_engine.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions (v_pk_*_f32) in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# roctx ranges (window solves, CG iterations, updates, operators)
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def _compile(hipcc, src, obj, verbose):
    cmd = [hipcc] + FLAGS + ["-c", "-I", os.path.join(ROOT, "include"),
                             "-I", os.path.join(HERE, "csrc"), "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o")
            for s in SOURCES]
    jobs = max(1, min(len(srcs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_compile, hipcc, s, o, verbose)
                  for s, o in zip(srcs, objs)]:
            f.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + ["-shared", "-o", tmp] + objs + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
