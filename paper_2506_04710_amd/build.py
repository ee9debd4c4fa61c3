"""Build the gfx950 shared library libtoeplitz.so in-tree with hipcc."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libtoeplitz.so")
SOURCES = ["tp_capi.hip", "tp_plan.hip", "tp_apply_f64.hip", "tp_apply_f32.hip", "tp_apply_wide.hip", "tp_gmres.hip",
           "tp_post.hip", "tp_mfma.hip", "tp_schur.hip", "tp_static.hip",
           "tp_tune.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # keep the compiler from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def _compile(src, verbose, extra, objdir=None):
    obj = os.path.join(objdir or OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra=(), out: str = OUT, objdir: str = OBJ, link_extra=()) -> str:
    """Compile every source and link libtoeplitz.so (or `out`); `extra` holds
    additional hipcc flags (e.g. -DTP_MFMA_MIN_R=8 to move the matrix-core
    threshold, or host-only sanitizer flags, each after -Xarch_host)."""
    os.makedirs(objdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, list(extra), objdir), SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *link_extra, *objs, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
