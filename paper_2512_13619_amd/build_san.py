"""Build a host-sanitised copy of libhdg.so for CPU-only checks of the C ABI.

The host code of every source (argument checks, workspace bookkeeping, the host spectral
helpers) is compiled with AddressSanitizer and UndefinedBehaviorSanitizer; the device code
is compiled as usual (no GPU sanitiser). The result, _build_san/libhdg_san.so, is loaded
by a process that preloads the ASan runtime (asan_runtime() gives its path), e.g.
    LD_PRELOAD=<runtime> ASAN_OPTIONS=detect_leaks=0 python -c "..."
It is a test build only: the product library is libhdg.so (build.py).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from .build import CSRC, HIPCC, ROOT, SOURCES

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build_san")
LIB = os.path.join(BUILD, "libhdg_san.so")
SAN = ["-Xarch_host", "-fsanitize=address",
       "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "-Wno-unknown-pragmas"]


def asan_runtime():
    """Path of the ASan runtime shared library of the ROCm clang."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + FLAGS + SAN + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r


def build():
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    for src, _, r in results:
        if r.returncode != 0:
            raise RuntimeError(f"sanitised build of {src} failed:\n{r.stdout}{r.stderr}")
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", LIB] + [o for _, o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitised link failed:\n" + r.stdout + r.stderr)
    return LIB


if __name__ == "__main__":
    sys.stdout.write(build() + "\n")
