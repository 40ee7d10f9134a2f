"""Build the CPU FP64 oracle (test infrastructure; never linked by the product).

    python oracle/build.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (-O1 -g), for the host-side checks; load it with libasan preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas", "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


def build(verbose: bool = False) -> str:
    # Generic x86-64 code: the library is built once and may run on another host.
    cmd = ["gcc", "-O3", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
