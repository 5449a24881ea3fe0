"""In-tree build of the native parts of the package.

* ``libpospopcnt.so``: the GPU library behind include/pospopcnt.h, compiled for
  gfx950 with hipcc (host code and kernels in one shared object).
* ``inputs/libppc_gen.so``: the seeded input generator, compiled with gcc.

Run ``python -m paper_1911_02696_amd.build``.  Every call recompiles.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpospopcnt.so")
GEN_SRC = os.path.join(PKG, "inputs", "ppc_gen.c")
GEN_LIB = os.path.join(PKG, "inputs", "libppc_gen.so")

ARCH = os.environ.get("PPC_OFFLOAD_ARCH", "gfx950")
HIP_SOURCES = ["ppc_single.hip", "ppc_batch.hip", "ppc_api.hip", "ppc_serve.hip",
               "ppc_onehot.hip", "ppc_wide.hip"]
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # Keep the compiler from emitting packed FP32 instructions anywhere.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise FileNotFoundError("hipcc not found")


def _replace(tmp: str, out: str):
    os.replace(tmp, out)


def build_gen() -> str:
    tmp = GEN_LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-pthread", "-shared",
                    "-fPIC", "-o", tmp, GEN_SRC], check=True)
    _replace(tmp, GEN_LIB)
    return GEN_LIB


def build_lib(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-o", tmp, *srcs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    _replace(tmp, LIB)
    return LIB


def build(verbose: bool = False):
    build_gen()
    build_lib(verbose=verbose)


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    print(GEN_LIB)
