"""Build ``libdeskew.so`` (HIP, gfx950) in-tree with hipcc.

Each source compiles to an object in parallel, then one link.
Usage: ``python -m paper_2211_00645_amd.build`` (or call ``build()``).

``--asan`` (``build(asan=True)``) builds ``libdeskew_asan.so`` instead: the
host code instrumented with AddressSanitizer (every ``-fsanitize=`` flag
goes to the host pass only; the device code is that of the normal build).
It is loaded with ``DSK_LIB`` pointing at it and the sanitizer runtime
preloaded, for host-only checks on a machine without a GPU.

``--bounds`` (``build(bounds=True)``) builds ``libdeskew_bounds.so``: the
debug build whose forward, batch and backward kernels check every global
address against its buffer's extent (``DSK_CHECK_BOUNDS=1``; read the count
with ``dsk_debug_bounds_violations``), loaded with ``DSK_LIB`` pointing at
it.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdeskew.so")
LIB_ASAN = os.path.join(PKG, "libdeskew_asan.so")
LIB_BOUNDS = os.path.join(PKG, "libdeskew_bounds.so")
SOURCES = ["deskew.hip", "batch.hip", "tune.hip", "rolling.hip", "view.hip", "affine.hip"]
ARCH = os.environ.get("DSK_OFFLOAD_ARCH", "gfx950")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument",
         "-I", INCLUDE, "-I", CSRC]


HOST_ASAN = "-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -Xarch_host -g".split()
HOST_ASAN_LINK = "-Xarch_host -fsanitize=address -shared-libasan".split()


def build(verbose: bool = False, asan: bool = False, bounds: bool = False) -> str:
    if asan and bounds:
        raise ValueError("one variant at a time")
    objdir = os.path.join(PKG, "_build", "asan" if asan else ("bounds" if bounds else ""))
    os.makedirs(objdir, exist_ok=True)
    lib = LIB_ASAN if asan else (LIB_BOUNDS if bounds else LIB)
    extra = HOST_ASAN if asan else (["-DDSK_CHECK_BOUNDS=1"] if bounds else [])

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc"] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    cmd = (["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC"] +
           (HOST_ASAN_LINK if asan else []) +
           ["-o", lib + ".tmp"] + objs)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def asan_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (to preload), or ''."""
    out = subprocess.run(["hipcc", "--print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else ""


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, asan="--asan" in sys.argv, bounds="--bounds" in sys.argv))
