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


SEG_LIMBS = 40   # 64-bit limbs per segment total written by bins.c


def _load_segmented():
    lib = _load()
    if not hasattr(lib, "_seg_ready"):
        lib.oracle_segmented_sums.restype = ctypes.c_int
        lib.oracle_segmented_sums.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        lib._seg_ready = True
    return lib


def segmented_exact_sums(buf, byte_offset, length, fmt_code, threads=None):
    """Exact states of many segments of one byte buffer.

    Segment i is length[i] elements of format fmt_code[i] (0 binary64,
    1 binary32, 2 bfloat16) starting byte_offset[i] bytes into buf (a numpy
    array, read as bytes).  Each segment is summed by the exponent bins of
    ``bins.c`` and folded there into one wide two's-complement integer, which
    becomes a Python int here.  Returns a list of ``ExactSum``.
    """
    raw = np.ascontiguousarray(np.asarray(buf).reshape(-1)).view(np.uint8)
    off = np.ascontiguousarray(byte_offset, dtype=np.uint64)
    ln = np.ascontiguousarray(length, dtype=np.uint64)
    fc = np.ascontiguousarray(fmt_code, dtype=np.uint32)
    nseg = len(off)
    if not (len(ln) == nseg and len(fc) == nseg):
        raise ValueError("segment arrays differ in length")
    esize = np.array([8, 4, 2], dtype=np.uint64)
    if nseg and (fc.max() > 2 or np.any(off + ln * esize[np.minimum(fc, 2)] > raw.size)):
        raise ValueError("segment outside the buffer or unknown format")
    limbs = np.zeros(nseg * SEG_LIMBS, dtype=np.uint64)
    special = np.zeros(max(nseg, 1), dtype=np.uint32)
    nthr = default_threads() if threads is None else int(threads)
    used = _load_segmented().oracle_segmented_sums(
        raw.ctypes.data if raw.size else None, off.ctypes.data, ln.ctypes.data,
        fc.ctypes.data, nseg, nthr, limbs.ctypes.data, special.ctypes.data)
    if used < 0:
        raise RuntimeError("oracle_segmented_sums rejected its arguments")
    data = limbs.tobytes()
    step = SEG_LIMBS * 8
    out = []
    sp = special.tolist()
    for i in range(nseg):
        total = int.from_bytes(data[i * step:(i + 1) * step], "little", signed=True)
        s = sp[i]
        out.append(ExactSum(total, bool(s & 1), bool(s & 2), bool(s & 4)))
    return out


def segmented_oracle_sums(buf, byte_offset, length, fmt_code, out_fmt=None,
                          threads=None):
    """Correctly rounded (RNE) result (bits, flags) of every segment; the
    output format defaults to binary64 for binary64 segments and binary32
    for the others."""
    names = ["f64", "f32", "f32"]
    accs = segmented_exact_sums(buf, byte_offset, length, fmt_code, threads)
    fc = np.asarray(fmt_code).tolist()
    return [tuple(finish(a, out_fmt or names[c])) for a, c in zip(accs, fc)]
