"""Build liblbm_hip.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["lbm_kernels.hip", "lbm_api.hip"]
LIB = os.path.join(HERE, "liblbm_hip.so")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-value",
]


HOST_SOURCES = ["lbm_fit.cpp", "lbm_tune.cpp"]   # host-only code (the LRS fit, the autotuner)
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall"]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-pthread", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


# Host-side sanitizer build: AddressSanitizer and UndefinedBehaviorSanitizer
# on the host code (the C ABI, argument validation, plan and arena layout,
# the LRS fit and the autotuner); the device code is compiled as usual, at
# -O1.  It serves the CPU-side tests.  Every sanitizer flag on a hipcc line
# sits behind -Xarch_host.
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]
SAN_HOST_FLAGS = ["-O1", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", "-pthread"]


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that a process loading the
    sanitized library must preload."""
    out = subprocess.check_output(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"])
    path = out.decode().strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return path


def build_sanitized(outdir: str, verbose: bool = False) -> str:
    """Build the host code of liblbm_hip.so with ASan + UBSan into outdir."""
    os.makedirs(outdir, exist_ok=True)
    xs = [a for f in SAN for a in ("-Xarch_host", f)]
    objs = []
    for src in SOURCES:
        obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", f"--offload-arch={ARCH}", *SAN_HOST_FLAGS, "-Xarch_host", "-g", *xs,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
        cmd = ["/opt/rocm/llvm/bin/clang++", *SAN_HOST_FLAGS, "-g", *SAN, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    lib = os.path.join(outdir, "liblbm_hip.so")
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-shared-libsan", *xs, "-pthread", "-o", lib, *objs,
           "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return lib


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(sys.argv[sys.argv.index("--sanitize") + 1], verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
