"""Build the HIP library libtalek_pir.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtalek_pir.so")
PROBE = os.path.join(HERE, "roofline_probe")  # measured HBM, VALU and LDS peaks
ARCH = os.environ.get("TALEK_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "xorpir_tile.hip",
    "xorpir_m4r.hip",
    "xorpir_m4rw.hip",
    "aux_kernels.hip",
    "plan.cpp",
    "pir_db.cpp",
    "cuckoo.cpp",
    "tune.cpp",
    "stream.cpp",
    "serve.cpp",
    "mask.hip",
    "iv_codec.hip",
    "strassen.hip",
    "noalloc.hip",
]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value", f"-I{os.path.join(ROOT, 'include')}"]
# Device code: gfx950 only; packed-FP32 instruction selection disabled.
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src: str, verbose: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = ["hipcc", *COMMON]
    if src.endswith(".hip"):
        cmd += DEVICE
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    cmd = ["hipcc", "-O3", "-std=c++17", "-Wall", *DEVICE, os.path.join(CSRC, "roofline_probe.hip"), "-o", PROBE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBE + ".tmp", PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
