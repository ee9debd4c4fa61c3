"""Compile the plain-C oracle into oracle/_oracle.so (gcc, OpenMP).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline load the result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
OUT = os.path.join(HERE, "_oracle.so")


def build(verbose: bool = False, sanitize: bool = False, out: str = OUT) -> str:
    """Compile oracle.c into `out`; sanitize: AddressSanitizer and
    UndefinedBehaviorSanitizer instrumentation (load with gcc's libasan
    preloaded)."""
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-O1" if sanitize else "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", *san,
           "-fno-fast-math", "-ffp-contract=off", "-fcx-fortran-rules", SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
