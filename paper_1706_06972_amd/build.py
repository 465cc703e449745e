"""Build libocsc.so (HIP, gfx950) in-tree.

    python -m paper_1706_06972_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libocsc.so")
SOURCES = [os.path.join(HERE, "csrc", "ocsc.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    # roctx ranges around the C-ABI calls
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
]


# Host-side AddressSanitizer / UndefinedBehaviorSanitizer build of the same
# source, for the C-ABI tests on the CPU (the device code is built as usual;
# each -fsanitize applies to the host compilation only).
LIB_SANITIZED = os.path.join(HERE, "_build_asan", "libocsc_asan.so")
SANITIZE_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-shared-libasan", "-g",
]


def asan_runtime() -> str:
    """Path of the shared ASan runtime that a sanitized library needs preloaded."""
    clang = os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang++")
    out = subprocess.run([clang, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True, check=True).stdout.strip()
    return out


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB_SANITIZED), exist_ok=True)
    tmp = LIB_SANITIZED + ".tmp"
    cmd = [HIPCC] + FLAGS + SANITIZE_FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_SANITIZED)
    return LIB_SANITIZED


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
