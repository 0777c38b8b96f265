"""Build the HIP shared library ``librks.so`` for gfx950 in-tree.

Every call recompiles: hipcc cross-compiles the device code without a GPU.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "librks.so")

ARCH = os.environ.get("RKS_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are kept out of the generated code on purpose.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-march=x86-64-v3", f"-I{INCLUDE}", f"-I{CSRC}"]

SOURCES = [
    ("kernels.hip", ["hipcc", "-x", "hip"] + HIP_FLAGS),
    ("net.hip", ["hipcc", "-x", "hip"] + HIP_FLAGS),
    ("rks_api.cpp", ["hipcc"] + HOST_FLAGS + ["-D__HIP_PLATFORM_AMD__"]),
    ("dense.cpp", ["g++"] + HOST_FLAGS),
    ("panels.cpp", ["g++"] + HOST_FLAGS),
]


def _compile(item):
    src, cmd = item
    obj = os.path.join(BUILD, src + ".o")
    full = cmd + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(full, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(full)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile all sources and link librks.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(link)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
