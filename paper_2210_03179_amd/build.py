"""Builds libsemcheb.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Usage: python -m paper_2210_03179_amd.build   (or call build()).
Object files go to paper_2210_03179_amd/_build/; the library is written next to
this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsemcheb.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "api.cpp", "host_setup.cpp", "batched.cpp"]
ARCH = os.environ.get("SEMCHEB_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-fopenmp", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fopenmp", f"--offload-arch={ARCH}", *objs, "-o", tmp,
           "-Wl,-rpath,/opt/rocm/lib/llvm/lib", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


# Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer: the
# setup, validation and host-array code (api.cpp, host_setup.cpp, batched.cpp) is compiled
# with the sanitizers on its host pass only; the device code is built as usual. The library
# expects the sanitizer runtime to be preloaded into the process (tests/test_host_sanitizers.py).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build_host_sanitized(out_dir: str) -> str:
    os.makedirs(out_dir, exist_ok=True)

    def comp(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        extra = SANITIZE if src != "kernels.hip" else []
        cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(comp, SOURCES))
    out = os.path.join(out_dir, "libsemcheb_sanitized.so")
    cmd = [HIPCC, "-shared", "-fopenmp", f"--offload-arch={ARCH}", *objs, "-o", out, *SANITIZE,
           "-Wl,-rpath,/opt/rocm/lib/llvm/lib", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking the sanitized library failed:\n{' '.join(cmd)}\n{r.stderr}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
