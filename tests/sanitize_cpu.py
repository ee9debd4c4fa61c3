"""Run the CPU test suite against sanitizer builds (not collected by pytest;
run as `python tests/sanitize_cpu.py [workdir]`, a few minutes).

Two passes, each in a process of its own:
  1. oracle.c built with gcc's AddressSanitizer and UndefinedBehaviorSanitizer
     (ORACLE_LIBRARY), gcc's libasan preloaded;
  2. the library's host code (C-ABI argument checks, layout and size
     accounting, host generator checks) built with clang's AddressSanitizer
     and UndefinedBehaviorSanitizer, host side only (device code as usual)
     (TOEPLITZ_LIBRARY), clang's ASan runtime preloaded.
A pass fails on a failing test or on any sanitizer report.  For CPU machines
only: where the environment already preloads a library, nothing is run."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

CLANG_RT = "/opt/rocm/lib/llvm/lib/clang"


def _clang_asan():
    for ver in sorted(os.listdir(CLANG_RT), reverse=True):
        p = os.path.join(CLANG_RT, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise FileNotFoundError("clang ASan runtime not found")


def _run(name, env_extra):
    env = dict(os.environ, **env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-x", "-q", "-m", "not gpu",
           "-p", "no:cacheprovider"]
    print(f"[sanitize] {name}: {' '.join(f'{k}={v}' for k, v in env_extra.items())}", flush=True)
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True)
    out = r.stdout + r.stderr
    reports = [l for l in out.splitlines() if "ERROR: AddressSanitizer" in l or "runtime error:" in l]
    tail = "\n".join(out.strip().splitlines()[-3:])
    print(tail, flush=True)
    ok = r.returncode == 0 and not reports
    if reports:
        print("\n".join(reports[:20]), flush=True)
    print(f"[sanitize] {name}: {'clean' if ok else 'FAILED'}", flush=True)
    return ok


def main(work):
    if os.environ.get("LD_PRELOAD") or os.path.exists("/etc/ld.so.preload"):
        # the passes preload a sanitizer runtime of their own; a machine that
        # already preloads a library is left as it is
        print("[sanitize] this environment already preloads a library; not run here", flush=True)
        return 0
    os.makedirs(work, exist_ok=True)
    from oracle import build as ob
    from paper_2506_04710_amd import build as lb
    orc = ob.build(sanitize=True, out=os.path.join(work, "_oracle_san.so"))
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    lib = lb.build(extra=san, out=os.path.join(work, "libtoeplitz_san.so"), objdir=os.path.join(work, "obj"))
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                              text=True).stdout.strip()
    ok1 = _run("oracle (gcc ASan+UBSan)", {"ORACLE_LIBRARY": orc, "LD_PRELOAD": gcc_asan})
    ok2 = _run("library host code (clang ASan+UBSan)", {"TOEPLITZ_LIBRARY": lib, "LD_PRELOAD": _clang_asan()})
    return 0 if ok1 and ok2 else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_build_sanitize")))
