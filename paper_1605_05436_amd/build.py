"""Build libxsum.so in-tree with hipcc for gfx950.

    python paper_1605_05436_amd/build.py   (runs without importing the package)
"""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libxsum.so")
SOURCES = ["xsum_kernels.hip", "xsum_segmented.hip", "xsum_plan.hip", "xsum_api.hip",
           "xsum_stream.hip", "xsum_state.hip"]
HEADERS = ["xsum_device.h", "xsum_internal.h", "xsum_segmented.h", "xsum_host.h"]
ARCH = os.environ.get("XSUM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # no packed-FP32 instructions are to be generated in any HIP code here
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep single-lane queue atomics as written: the optimiser's rewrite reads
    # the result back at once, which would serialise the pop of the next work
    # item with the current one instead of overlapping them
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose=False):
    """Compile every HIP source into libxsum.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I" + INCLUDE, "-I" + CSRC] + \
        [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                         text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "--hip-link" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
