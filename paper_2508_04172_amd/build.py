"""Builds the in-tree HIP library ``librbfl.so`` for gfx950 with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
generation disabled, and linked against rocSOLVER/rocBLAS (start-up stage
SVD and LU).  Usage: ``python -m paper_2508_04172_amd.build`` (``--sanitize``
for the host-sanitized variant).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librbfl.so")
SOURCES = ["rbfl_host.hip", "rbfl_eval.hip", "surrogate_host.hip", "rbfl_query.hip", "host_math.hip", "rbfl_plan.hip", "sampler_host.hip", "rbfl_store.hip", "rbfl_static.hip", "build_kernels.hip", "eval_kernels.hip", "contract_fp64.hip",
           "contract_split.hip", "contract_bf16.hip", "brute.hip", "mlp.hip", "sampler.hip"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{ROCM}/include",
]


def _hipcc() -> str:
    p = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer variant
# (librbfl_san.so): the same sources with the sanitizers on the host
# compilation only (device code unchanged), for CPU-only checks of the host
# logic (spec validation, store parsing, argument checks) under the clang
# ASan runtime.  Each sanitizer flag is scoped to the host pass.
LIB_SAN = os.path.join(HERE, "librbfl_san.so")
OUT_DIR_SAN = os.path.join(HERE, "_build_san")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def asan_runtime() -> str:
    """The clang ASan runtime the sanitized variant links against (preloaded
    into an uninstrumented interpreter)."""
    r = subprocess.run([os.path.join(ROCM, "lib", "llvm", "bin", "clang"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    return r.stdout.strip()


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out_dir, lib = (OUT_DIR_SAN, LIB_SAN) if sanitize else (OUT_DIR, LIB)
    extra = ["-O1", "-g", *SAN_FLAGS] if sanitize else []
    os.makedirs(out_dir, exist_ok=True)
    hipcc = _hipcc()
    objs = []

    def compile_one(src):
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        err = _run([hipcc, *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose and err.strip():
            print(err, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp"
    link_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan"] \
        if sanitize else []
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *link_san, "-o", tmp, *objs,
          f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
