"""Build the HIP library libpsfm.so for gfx950 (hipcc, in-tree).

Each source is compiled to an object in parallel (every kernel is launched
from the file that defines it), then the objects are linked."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
SOURCES = ["context.hip", "fit.hip", "solve.hip", "convolve.hip", "batch.hip", "cnn.hip",
           "noalloc.hip", "noise.hip", "stack.hip"]
LIB = os.path.join(PKG, "libpsfm.so")
OBJDIR = os.path.join(ROOT, "_build")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions stay off (plain FP32 FMA only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-pass-failed",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, s.replace(".hip", ".o"))
        jobs.append((["hipcc", *FLAGS, *inc, "-c", "-o", obj, os.path.join(HERE, s)], obj))

    def run(job):
        cmd, _ = job
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    workers = min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(run, jobs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for _, o in jobs]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
