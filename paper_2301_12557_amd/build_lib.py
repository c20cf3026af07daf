"""Build libfcfc.so (the gfx950 HIP library) in-tree with hipcc.

Flags: gfx950 only; -O3; -ffp-contract=off so that only the explicit fmaf
calls of the FP32 path fuse and the FP64 edge recheck rounds every operation
separately; packed-FP32 instructions disabled for the device code.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUTDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUTDIR, "libfcfc.so")
SOURCES = ["plan.cpp", "api.cpp", "mem.cpp", "build.hip", "worklist.hip", "tree.hip", "count.hip", "batch.hip", "mlp.hip", "tune.cpp",
           "diag.hip", "estimators.hip", "angular.hip", "binning.hip", "triplets.hip", "noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OUTDIR, src + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC, *FLAGS, *lang, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(OUTDIR, exist_ok=True)
    srcs = list(SOURCES)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
