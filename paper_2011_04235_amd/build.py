"""Builds libfastpi.so (HIP kernels for gfx950 + host library) in this directory."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfastpi.so")
SOURCES = ["api.cpp", "driver.cpp", "reorder.cpp", "plan.cpp", "rank_alloc.cpp", "block_svd.hip", "eig.hip", "dense.hip",
           "sparse.hip", "mlp.hip", "pchol.hip", "evaluate.hip", "randomized.hip", "reorder_gpu.hip", "subspace.hip", "mfma_gemm.hip"]
ARCH = "gfx950"
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Host-sanitizer build (libfastpi_san.so): AddressSanitizer and UndefinedBehaviorSanitizer on
# the host half of every source only (device code is built as usual), against the shared
# sanitizer runtime so that the library can be loaded into an uninstrumented Python with that
# runtime preloaded.
SAN_OUT = os.path.join(HERE, "libfastpi_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-shared-libasan", "-g"]


def _compile(src: str, obj_dir: str, extra=()) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    obj_dir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    out = SAN_OUT if sanitize else OUT
    extra = SAN_FLAGS if sanitize else ()
    os.makedirs(obj_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir, extra), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def sanitizer_runtime() -> str:
    """Path of the shared AddressSanitizer runtime the sanitizer build links against."""
    res = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


if __name__ == "__main__":
    if "--sanitizer-runtime" in sys.argv:
        print(sanitizer_runtime())
    else:
        build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
