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
           "xsum_truncated.hip",
           "xsum_stream.hip", "xsum_state.hip", "xsum_probe.hip"]
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


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                         text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "--hip-link" not in l)
    return res.returncode, out


def build(verbose=False):
    """Compile every HIP source into libxsum.so (always recompiles).  The
    sources are compiled to objects in parallel, then linked."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(ROOT, "_build", "xsum.%d" % os.getpid())
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        jobs.append((obj, [hipcc()] + compile_flags + ["-I" + INCLUDE, "-I" + CSRC, "-c",
                                                       os.path.join(CSRC, src), "-o", obj]))
    workers = min(len(jobs), max(1, os.cpu_count() or 1), 8)
    with ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(lambda j: _run(j[1]), jobs))
    for (obj, cmd), (rc, out) in zip(jobs, results):
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            raise RuntimeError("hipcc failed:\n" + out)
        if verbose and out.strip():
            print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + \
        [obj for obj, _ in jobs] + ["-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, out = _run(link)
    if rc != 0:
        raise RuntimeError("hipcc link failed:\n" + out)
    os.replace(tmp, LIB)
    for obj, _ in jobs:
        os.remove(obj)
    os.rmdir(objdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
