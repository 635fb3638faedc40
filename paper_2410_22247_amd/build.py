"""Build libaaqaoa.so (HIP, gfx950) in the package directory with hipcc.

Every translation unit (the common kernels, one per (precision, tile size)
instantiation of the sweep engine, the host code) is compiled to an object in
parallel, then the objects are linked into the shared library.
"""
import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaaqaoa.so")


def sources():
    return ([os.path.join(CSRC, "aaq_kernels.hip"), os.path.join(CSRC, "aaq_noalloc.hip")]
            + sorted(glob.glob(os.path.join(CSRC, "aaq_inst_*.hip")))
            + [os.path.join(CSRC, "aaq_host.cpp"), os.path.join(CSRC, "aaq_orbits.cpp")])


# Packed FP32 instructions are disabled for all device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _clean(stderr: str) -> str:
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


# Host-side sanitizer build (CPU checks of validation, planning and the orbit code): the
# host half of every translation unit instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer, device code untouched; the runtime is preloaded into the
# process (libclang_rt.asan of the ROCm clang), so the link line names no sanitizer.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
LIB_HOST_SANITIZE = os.path.join(ROOT, "_build", "libaaqaoa_hostsan.so")  # outside the package: CPU checks only


def build(verbose: bool = False, jobs: int = 0, host_sanitize: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = sources()
    flags = FLAGS + (HOST_SANITIZE if host_sanitize else [])
    lib = LIB_HOST_SANITIZE if host_sanitize else LIB
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="aaq_build_") as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [hipcc] + flags + ["-x", "hip", "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, r.returncode, _clean(r.stderr)

        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(compile_one, srcs))
        for src, _, rc, err in results:
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{err}")
            if verbose and err.strip():
                print(err, file=sys.stderr)
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for _, o, _, _ in results] + ["-o", lib + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + _clean(r.stderr))
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, host_sanitize="--host-sanitize" in sys.argv))
