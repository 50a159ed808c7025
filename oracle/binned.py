"""Multithreaded exact sum for large inputs: exponent bins in C, folded into
one Python int here.

TEST INFRASTRUCTURE ONLY (see the package docstring).

``bins.c`` adds each input's signed integer significand into a 128-bit bin
selected by its biased exponent.  The exact sum (Section 2 of the paper: a
wide fixed-point integer) is then sum_E bin[E] * 2^q(E), with q(E) the scale
of exponent E in units of 2^-1074 as defined by ``ieee.decode``.  The
decomposition (per-exponent bins, no shifting in the loop) is deliberately
unlike any GPU digit layout.
"""

import ctypes
import os
import subprocess
import threading

import numpy as np

from .exact import ExactSum, finish
from .ieee import FORMATS, fmt_of, decode

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bins.c")
_LIB = os.path.join(_HERE, "_oracle_bins.so")
_FMT_CODE = {"f64": 0, "f32": 1, "bf16": 2}
_lock = threading.Lock()
_lib = None


def build_binned(force=True):
    """Compile bins.c into _oracle_bins.so next to it (gcc, -O2, pthreads)."""
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC",
                           "-pthread", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or \
                    os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build_binned()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_binned_sum.restype = ctypes.c_int
            lib.oracle_binned_sum.argtypes = [
                ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                ctypes.c_void_p, ctypes.c_void_p]
            _lib = lib
    return _lib


def default_threads():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def exact_sum_binned(x, fmt, threads=None):
    """Exact state (``ExactSum``) of the inputs x of format fmt.

    x: numpy array of floats or of their bit patterns (any shape; it is read
    contiguously).  Returns (ExactSum, threads_used).
    """
    f = fmt_of(fmt)
    dt = {64: np.uint64, 32: np.uint32, 16: np.uint16}[f.width]
    a = np.ascontiguousarray(np.asarray(x).view(dt).reshape(-1))
    bins = np.zeros(2 * 2048, dtype=np.int64)
    special = np.zeros(1, dtype=np.uint32)
    nthr = default_threads() if threads is None else int(threads)
    used = _load().oracle_binned_sum(
        a.ctypes.data if a.size else None, a.size, _FMT_CODE[f.name], nthr,
        bins.ctypes.data, special.ctypes.data)
    if used < 0:
        raise RuntimeError("oracle_binned_sum rejected its arguments")
    # bins.c widens bfloat16 to binary32 (exact), so its bins are binary32's
    g = FORMATS["f32"] if f.name == "bf16" else f
    total = 0
    lo = bins[0::2].view(np.uint64).tolist()
    hi = bins[1::2].tolist()
    for e in range(g.emax_field):
        v = (hi[e] << 64) | lo[e]
        if v:
            # scale of biased exponent e: that of the pattern with this
            # exponent field and an empty mantissa field
            _, _, _, q = decode(e << g.t, g)
            total += v << q
    sp = int(special[0])
    return ExactSum(total, bool(sp & 1), bool(sp & 2), bool(sp & 4)), used


def oracle_sum_binned(x, fmt, out_fmt=None, threads=None):
    """Correctly rounded (RNE) sum of x; see ``exact.oracle_sum``."""
    f = fmt_of(fmt)
    if out_fmt is None:
        out_fmt = "f32" if f.name == "bf16" else f.name
    acc, _ = exact_sum_binned(x, f, threads)
    return finish(acc, out_fmt)
