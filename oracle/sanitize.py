"""CPU sanitizer runs (test infrastructure; no GPU involved).

    python oracle/sanitize.py [oracle] [host] [tsan]

oracle  the FP64 oracle built with gcc -fsanitize=address,undefined (_build/liboracle_asan.so)
        and the whole ``-m "not gpu"`` tier run against it (ORACLE_LIB), gcc's ASan runtime
        preloaded into the Python process.
host    the HIP library with its host code instrumented (AddressSanitizer and
        UndefinedBehaviorSanitizer on the host half of every translation unit: validation,
        planning, workspace layout, orbits, eta_p; device code unchanged), built by
        ``paper_2410_22247_amd/build.py --host-sanitize``, and the same tier run against it
        (AAQAOA_LIB) with the ROCm clang ASan runtime preloaded.  The GPU entry points fail
        on this machine after validation, so what runs is every host path the CPU tests reach.
tsan    the OpenMP oracle under ThreadSanitizer: oracle/tsan_check.c and qaoa_oracle.c built
        with the ROCm clang (-fsanitize=thread -fopenmp, the OpenMP runtime's Archer tool
        makes its synchronisation visible), run with several threads, each result compared
        with the one-thread result.

Every run stops at the first report (halt_on_error).  Exit status 0 = all requested runs clean.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build")
ROCM_LLVM = "/opt/rocm/llvm"


def _run(cmd, env=None):
    print("+", " ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


def _env(**kw):
    e = dict(os.environ)
    e.update({k: str(v) for k, v in kw.items()})
    return e


def _pytest():
    return [sys.executable, "-m", "pytest", "tests", "-q", "-m", "not gpu", "-p", "no:cacheprovider", "-n", "4"]


def oracle_asan() -> int:
    lib = os.path.join(OUT, "liboracle_asan.so")
    rc = _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
               "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", os.path.join(HERE, "qaoa_oracle.c"), "-o", lib,
               "-lm"])
    if rc:
        return rc
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return _run(_pytest(), _env(LD_PRELOAD=rt, ORACLE_LIB=lib, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))


def host_asan() -> int:
    sys.path.insert(0, ROOT)
    from paper_2410_22247_amd import build as B

    lib = B.build(verbose=False, host_sanitize=True)
    rts = sorted(glob.glob(os.path.join(ROCM_LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not rts:
        print("no clang ASan runtime found", file=sys.stderr)
        return 1
    return _run(_pytest(), _env(LD_PRELOAD=rts[-1], AAQAOA_LIB=lib, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))


def oracle_tsan() -> int:
    exe = os.path.join(OUT, "oracle_tsan_check")
    rc = _run([os.path.join(ROCM_LLVM, "bin", "clang"), "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=thread",
               os.path.join(HERE, "tsan_check.c"), os.path.join(HERE, "qaoa_oracle.c"), "-o", exe, "-lm",
               "-Wl,-rpath," + os.path.join(ROCM_LLVM, "lib")])
    if rc:
        return rc
    return _run([exe], _env(OMP_TOOL_LIBRARIES=os.path.join(ROCM_LLVM, "lib", "libarcher.so"), OMP_NUM_THREADS=4,
                           TSAN_OPTIONS="halt_on_error=1 ignore_noninstrumented_modules=1"))


if __name__ == "__main__":
    os.makedirs(OUT, exist_ok=True)
    which = sys.argv[1:] or ["oracle", "host", "tsan"]
    rc = 0
    for w in which:
        r = {"oracle": oracle_asan, "host": host_asan, "tsan": oracle_tsan}[w]()
        print(f"{w}: {'clean' if r == 0 else 'FAILED (%d)' % r}", flush=True)
        rc = rc or r
    sys.exit(rc)
