"""Build the native libraries for gfx950 in-tree.

    python -m paper_2608_16960_amd.build [-v]

libtsp.so   projector (include/tsp.h): csrc/tsp_*.hip
libtspnn.so companions of the learned and differentiable paths (include/tspnn.h):
            csrc/nn_*.hip
Objects go to _build/ (not committed); the .so files land next to this file.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OBJ = os.path.join(ROOT, "_build")
ARCH = os.environ.get("TSP_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # arithmetic is exactly what the source says: the count and fill passes of
    # the tracer re-evaluate the same expressions and must agree bit for bit
    "-ffp-contract=off",
    # hardware float atomics for the atomic adjoint
    "-munsafe-fp-atomics",
    # never emit packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", INC, "-I", CSRC,
]

LIBS = {
    "libtsp.so": "tsp_*.hip",
    "libtspnn.so": "nn_*.hip",
}


def _compile(src, verbose):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if verbose and (r.stderr.strip()):
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False):
    os.makedirs(OBJ, exist_ok=True)
    out = []
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        jobs = {}
        for lib, pat in LIBS.items():
            srcs = sorted(glob.glob(os.path.join(CSRC, pat)))
            if srcs:
                jobs[lib] = [ex.submit(_compile, s, verbose) for s in srcs]
        for lib, futs in jobs.items():
            objs = [f.result() for f in futs]
            target = os.path.join(PKG, lib)
            cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", target + ".tmp",
                   *objs]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            os.replace(target + ".tmp", target)
            out.append(target)
    return out


if __name__ == "__main__":
    for p in build(verbose="-v" in sys.argv):
        print(p)
