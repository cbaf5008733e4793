"""Build libtor.so (the HIP kernels and the C ABI) for gfx950, in-tree.

``python -m paper_2109_04528_amd.build`` compiles the HIP sources in
``csrc/`` (the recursive, comparison, staging, subset-sum and probe kernels)
and ``csrc/tor_runtime.cpp`` with hipcc into ``paper_2109_04528_amd/libtor.so``.
Packed-FP32 instructions are disabled; no fast-math (the double-double
accumulation relies on IEEE rounding and no reassociation).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtor.so")
ARCH = os.environ.get("TOR_OFFLOAD_ARCH", "gfx950")

SOURCES = ["tor_kernels.hip", "tor_compare.hip", "tor_stage.hip", "tor_zeta.hip", "tor_probe.hip", "tor_runtime.cpp"]
# the double-double factor's kernel: its own translation unit, compiled with
# the AMDGPU scheduler's register-pressure trackers, which schedule it about
# 4 % faster (the FP64 kernels gain nothing from them)
QUAD_SOURCE = "tor_kernels_quad.hip"
QUAD_FLAGS = ["-mllvm", "-amdgpu-use-amdgpu-trackers"]
OBJ_DIR = os.path.join(HERE, "_build")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def build(verbose: bool = False, extra=None) -> str:
    common = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-fno-fast-math", "-Wall", "-Wno-unused-function",
              "-I", os.path.join(HERE, "..", "include")]
    os.makedirs(OBJ_DIR, exist_ok=True)
    quad_obj = os.path.join(OBJ_DIR, "tor_kernels_quad.o")
    qcmd = common + QUAD_FLAGS + ["-c", "-x", "hip", os.path.join(CSRC, QUAD_SOURCE), "-o", quad_obj] + \
        list(extra or [])
    cmd = common + ["-shared", "-x", "hip"] + [os.path.join(CSRC, s) for s in SOURCES] + \
        ["-x", "none", quad_obj, "-o", LIB + ".tmp", "-lpthread"] + list(extra or [])
    for c in (qcmd, cmd):
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.run(c, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


SAN_DIR = os.path.join(HERE, "san")
SAN_LIB = os.path.join(SAN_DIR, "libtor_san.so")
SAN_EXE = os.path.join(SAN_DIR, "runtime_sanitized")


def build_sanitized(verbose: bool = False) -> str:
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    on its host code (each -fsanitize after -Xarch_host, so the kernels are
    the usual ones), and the C driver of tests/runtime_sanitize_main.c that
    calls every entry point through it."""
    os.makedirs(SAN_DIR, exist_ok=True)
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O2", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-fno-fast-math", "-Wno-unused-function"] + san + \
          ["-I", os.path.join(HERE, "..", "include"), "-x", "hip"] + \
          [os.path.join(CSRC, s) for s in SOURCES + [QUAD_SOURCE]] + ["-o", SAN_LIB + ".tmp", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    drv = [clang, "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(HERE, "..", "include"),
           os.path.join(HERE, "..", "tests", "runtime_sanitize_main.c"),
           "-L", SAN_DIR, "-ltor_san", "-Wl,-rpath,$ORIGIN", "-lm", "-o", SAN_EXE]
    if verbose:
        print(" ".join(drv), flush=True)
    subprocess.run(drv, check=True)
    return SAN_EXE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
