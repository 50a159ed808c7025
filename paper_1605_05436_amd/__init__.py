"""Python binding of libxsum: exact floating-point summation on MI355X.

Argument marshalling only: every step of a sum runs in the HIP library
(libxsum.so, built from csrc/ by ``build.py``).  If the library is missing the
import of this module fails; there is no fallback.

The C names are kept: ``xsum_exact_sum``, ``xsum_exact_sum_async``,
``xsum_exact_sum_async_blocks``, ``xsum_acc_zero``, ``xsum_acc_add``,
``xsum_acc_merge``, ``xsum_acc_finalize``, ``xsum_last_error``.  They take raw
device pointers (ints) and a stream handle (int, 0 = default stream).  The
helpers ``exact_sum``, ``new_states`` and ``stream_handle`` accept PyTorch
tensors, which serve only as device memory and streams.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxsum.so")

F64, F32, BF16, SAME = 0, 1, 2, 255
OK, EINVAL, EDTYPE, ENOMEM, EHIP, ERANGE = 0, 1, 2, 3, 4, 5
FLAG_INEXACT, FLAG_OVERFLOW, FLAG_NAN, FLAG_INF = 1, 2, 4, 8
DIGITS = 68
STATE_BYTES = 576
TUNE_BUCKETS = 24
OUT_BYTES = {F64: 8, F32: 4, BF16: 2}

EXPORTED = [
    "xsum_version", "xsum_last_error", "xsum_exact_sum", "xsum_exact_sum_f64",
    "xsum_exact_sum_async", "xsum_exact_sum_async_blocks", "xsum_acc_zero",
    "xsum_acc_add", "xsum_acc_merge", "xsum_acc_finalize",
    "xsum_acc_add_host", "xsum_exact_sum_host", "xsum_state_encode",
    "xsum_state_decode",
    "xsum_segmented_plan", "xsum_plan_destroy", "xsum_plan_get_info",
    "xsum_plan_workspace_size", "xsum_segmented_workspace_size",
    "xsum_exact_sum_segmented", "xsum_segmented_workspace_init",
    "xsum_segmented_run", "xsum_segmented_run_noalloc", "xsum_segmented_capture", "xsum_graph_launch",
    "xsum_graph_destroy", "xsum_batch_item_tasks", "xsum_batch_add",
    "xsum_batch_finalize", "xsum_probe_read", "xsum_probe_flush", "xsum_probe_clock",
    "xsum_truncated_workspace_size", "xsum_truncated_round",
    "xsum_exact_sum_truncated",
]

# xsum_batch_item_t as a numpy record (32 bytes)
def batch_item_dtype():
    import numpy as np
    return np.dtype([("ptr", "<u8"), ("length", "<u8"), ("dtype", "<u4"),
                     ("slot", "<u4"), ("first_task", "<u8")])


class SegTuning(ctypes.Structure):
    """xsum_seg_tuning_t (0 = library default in every field)."""
    _fields_ = [("lane_max", ctypes.c_uint64 * 3), ("wave_max", ctypes.c_uint64 * 3),
                ("chunk_vectors", ctypes.c_uint64),
                ("blocks_per_cu", ctypes.c_uint32), ("lane_buckets", ctypes.c_uint32),
                ("two_lanes_from", ctypes.c_uint64), ("four_lanes_from", ctypes.c_uint64),
                ("lanes", (ctypes.c_uint8 * TUNE_BUCKETS) * 3),
                ("lane_unroll", (ctypes.c_uint8 * TUNE_BUCKETS) * 3)]


TRUNC_MAX_R = 16


class TruncRoot(ctypes.Structure):
    """xsum_trunc_root_t: the root of one truncated pass."""
    _fields_ = [("index", ctypes.c_int32 * TRUNC_MAX_R),
                ("value", ctypes.c_int64 * TRUNC_MAX_R),
                ("count", ctypes.c_uint32), ("bound_index", ctypes.c_int32),
                ("bound_value", ctypes.c_uint64), ("special", ctypes.c_uint32),
                ("certified", ctypes.c_uint32), ("bits", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("r", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    """xsum_plan_info_t."""
    _fields_ = [("nseg", ctypes.c_uint64), ("lane_segments", ctypes.c_uint64),
                ("wave_segments", ctypes.c_uint64),
                ("chunked_segments", ctypes.c_uint64), ("chunks", ctypes.c_uint64),
                ("work_items", ctypes.c_uint64), ("lane_max", ctypes.c_uint64 * 3),
                ("wave_max", ctypes.c_uint64 * 3),
                ("chunk_vectors", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("blocks", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class XsumError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("xsum status %d: %s" % (status, message))
        self.status = status


def _hip_runtimes_loaded():
    """Distinct libamdhip64 files mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as f:
            maps = f.read()
    except OSError:
        return []
    found = set()
    for line in maps.splitlines():
        path = line.split()[-1] if line.split() else ""
        if os.path.basename(path).startswith("libamdhip64.so"):
            found.add(os.path.realpath(path))
    return sorted(found)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libxsum.so is not built (expected at %s); run "
            "`python paper_1605_05436_amd/build.py`" % LIB_PATH)
    # The library must run on the same HIP runtime as the PyTorch tensors it
    # is handed.  PyTorch ships its own libamdhip64.so.7; loading torch first
    # lets the dynamic loader bind libxsum's dependency of that soname to the
    # copy already in the process instead of loading a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_loaded()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are loaded in this process (%s); "
                          "libxsum would not see the same devices and memory "
                          "as PyTorch" % ", ".join(runtimes))
    vp, u64, i32, u32p = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, \
        ctypes.POINTER(ctypes.c_uint32)
    lib.xsum_version.restype = ctypes.c_char_p
    lib.xsum_version.argtypes = []
    lib.xsum_last_error.restype = ctypes.c_char_p
    lib.xsum_last_error.argtypes = []
    lib.xsum_exact_sum.restype = i32
    lib.xsum_exact_sum.argtypes = [vp, u64, i32, i32, vp, u32p, vp]
    lib.xsum_exact_sum_f64.restype = ctypes.c_double
    lib.xsum_exact_sum_f64.argtypes = [vp, u64, i32]
    lib.xsum_exact_sum_async.restype = i32
    lib.xsum_exact_sum_async.argtypes = [vp, u64, i32, i32, vp, vp, vp, vp]
    lib.xsum_exact_sum_async_blocks.restype = i32
    lib.xsum_exact_sum_async_blocks.argtypes = [vp, u64, i32, i32, vp, vp, vp,
                                                i32, vp]
    lib.xsum_acc_zero.restype = i32
    lib.xsum_acc_zero.argtypes = [vp, u64, vp]
    lib.xsum_acc_add.restype = i32
    lib.xsum_acc_add.argtypes = [vp, vp, u64, i32, vp]
    lib.xsum_acc_merge.restype = i32
    lib.xsum_acc_merge.argtypes = [vp, vp, vp]
    lib.xsum_acc_finalize.restype = i32
    lib.xsum_acc_finalize.argtypes = [vp, i32, vp, vp, vp]
    lib.xsum_acc_add_host.restype = i32
    lib.xsum_acc_add_host.argtypes = [vp, vp, u64, i32, u64, vp]
    lib.xsum_exact_sum_host.restype = i32
    lib.xsum_exact_sum_host.argtypes = [vp, u64, i32, i32, vp, u32p, u64, vp]
    lib.xsum_state_encode.restype = i32
    lib.xsum_state_encode.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.xsum_state_decode.restype = i32
    lib.xsum_state_decode.argtypes = [vp, ctypes.c_size_t, vp]
    lib.xsum_segmented_plan.restype = i32
    lib.xsum_segmented_plan.argtypes = [vp, u64, i32, vp, ctypes.POINTER(vp)]
    lib.xsum_plan_destroy.restype = None
    lib.xsum_plan_destroy.argtypes = [vp]
    lib.xsum_plan_get_info.restype = i32
    lib.xsum_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.xsum_plan_workspace_size.restype = ctypes.c_size_t
    lib.xsum_plan_workspace_size.argtypes = [vp]
    lib.xsum_segmented_workspace_size.restype = ctypes.c_size_t
    lib.xsum_segmented_workspace_size.argtypes = [u64, u64]
    lib.xsum_exact_sum_segmented.restype = i32
    lib.xsum_exact_sum_segmented.argtypes = [vp, vp, u64, i32, vp, vp, vp,
                                             ctypes.c_size_t, vp]
    lib.xsum_segmented_workspace_init.restype = i32
    lib.xsum_segmented_workspace_init.argtypes = [vp, ctypes.c_size_t, vp]
    lib.xsum_segmented_run.restype = i32
    lib.xsum_segmented_run.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.xsum_segmented_run_noalloc.restype = i32
    lib.xsum_segmented_run_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.xsum_segmented_capture.restype = i32
    lib.xsum_segmented_capture.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t,
                                           ctypes.POINTER(vp)]
    lib.xsum_graph_launch.restype = i32
    lib.xsum_graph_launch.argtypes = [vp, vp]
    lib.xsum_graph_destroy.restype = None
    lib.xsum_graph_destroy.argtypes = [vp]
    lib.xsum_batch_item_tasks.restype = u64
    lib.xsum_batch_item_tasks.argtypes = [u64, u64, i32, u64]
    lib.xsum_batch_add.restype = i32
    lib.xsum_batch_add.argtypes = [vp, ctypes.c_uint32, u64, u64, vp, vp, vp]
    lib.xsum_batch_finalize.restype = i32
    lib.xsum_batch_finalize.argtypes = [vp, vp, ctypes.c_uint32, vp, vp, vp, vp]
    lib.xsum_probe_read.restype = i32
    lib.xsum_probe_read.argtypes = [vp, u64, vp, vp]
    lib.xsum_probe_flush.restype = i32
    lib.xsum_probe_flush.argtypes = [vp, u64, ctypes.c_uint32, vp]
    lib.xsum_probe_clock.restype = i32
    lib.xsum_probe_clock.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, vp]
    lib.xsum_truncated_workspace_size.restype = ctypes.c_size_t
    lib.xsum_truncated_workspace_size.argtypes = []
    lib.xsum_truncated_round.restype = i32
    lib.xsum_truncated_round.argtypes = [vp, u64, i32, i32, i32, vp, vp, ctypes.c_size_t, vp]
    lib.xsum_exact_sum_truncated.restype = i32
    lib.xsum_exact_sum_truncated.argtypes = [vp, u64, i32, i32, vp, u32p,
                                             ctypes.POINTER(ctypes.c_int), vp,
                                             ctypes.c_size_t, vp]
    return lib


_lib = _load()


def _check(status):
    if status != OK:
        raise XsumError(status, xsum_last_error())


def _p(x):
    return ctypes.c_void_p(int(x)) if x else None


def xsum_version():
    return _lib.xsum_version().decode()


def xsum_last_error():
    return _lib.xsum_last_error().decode()


def xsum_exact_sum(x, n, dtype, out_dtype=SAME, stream=0):
    """Blocking exact sum of n elements at device address x.
    Returns (result bit pattern as int, flags)."""
    out = ctypes.c_uint64(0)
    flags = ctypes.c_uint32(0)
    _check(_lib.xsum_exact_sum(_p(x), n, dtype, out_dtype, ctypes.byref(out),
                               ctypes.byref(flags), _p(stream)))
    ob = OUT_BYTES[(F64 if dtype == F64 else F32) if out_dtype == SAME else out_dtype]
    return out.value & ((1 << (8 * ob)) - 1), flags.value


def xsum_exact_sum_f64(x, n, dtype):
    return _lib.xsum_exact_sum_f64(_p(x), n, dtype)


def xsum_exact_sum_async(x, n, dtype, out_dtype, out, flags, scratch, stream=0):
    _check(_lib.xsum_exact_sum_async(_p(x), n, dtype, out_dtype, _p(out),
                                     _p(flags), _p(scratch), _p(stream)))


def xsum_exact_sum_async_blocks(x, n, dtype, out_dtype, out, flags, scratch,
                                blocks, stream=0):
    _check(_lib.xsum_exact_sum_async_blocks(_p(x), n, dtype, out_dtype, _p(out),
                                            _p(flags), _p(scratch), blocks,
                                            _p(stream)))


def xsum_acc_zero(acc, count, stream=0):
    _check(_lib.xsum_acc_zero(_p(acc), count, _p(stream)))


def xsum_acc_add(acc, x, n, dtype, stream=0):
    _check(_lib.xsum_acc_add(_p(acc), _p(x), n, dtype, _p(stream)))


def xsum_acc_merge(dst, src, stream=0):
    _check(_lib.xsum_acc_merge(_p(dst), _p(src), _p(stream)))


def xsum_acc_finalize(acc, out_dtype, out, flags, stream=0):
    _check(_lib.xsum_acc_finalize(_p(acc), out_dtype, _p(out), _p(flags),
                                  _p(stream)))


def xsum_acc_add_host(acc, x_host, n, dtype, chunk_bytes=0, stream=0):
    _check(_lib.xsum_acc_add_host(_p(acc), _p(x_host), n, dtype, chunk_bytes,
                                  _p(stream)))


def xsum_exact_sum_host(x_host, n, dtype, out_dtype=SAME, chunk_bytes=0, stream=0):
    """Blocking exact sum of n elements at host address x_host, streamed
    through the device in chunks.  Returns (result bit pattern, flags)."""
    out = ctypes.c_uint64(0)
    flags = ctypes.c_uint32(0)
    _check(_lib.xsum_exact_sum_host(_p(x_host), n, dtype, out_dtype, ctypes.byref(out),
                                    ctypes.byref(flags), chunk_bytes, _p(stream)))
    ob = OUT_BYTES[(F64 if dtype == F64 else F32) if out_dtype == SAME else out_dtype]
    return out.value & ((1 << (8 * ob)) - 1), flags.value


def exact_sum_host(array, dtype, out_dtype=SAME, chunk_bytes=0, stream=None):
    """Blocking exact sum of a contiguous host array (numpy array or CPU
    tensor; raw bit patterns are fine) of library dtype `dtype`.
    Returns (result bit pattern, flags)."""
    if hasattr(array, "data_ptr"):
        if array.is_cuda or not array.is_contiguous():
            raise ValueError("a contiguous CPU tensor is required")
        ptr, nbytes = array.data_ptr(), array.numel() * array.element_size()
    else:
        if not array.flags["C_CONTIGUOUS"]:
            raise ValueError("a C-contiguous array is required")
        ptr, nbytes = array.ctypes.data, array.nbytes
    n = nbytes // {F64: 8, F32: 4, BF16: 2}[dtype]
    return xsum_exact_sum_host(ptr, n, dtype, out_dtype, chunk_bytes,
                               stream_handle(stream) if stream is not None else 0)


STATE_ENCODED_MAX = 292


def xsum_state_encode(state):
    """Compact encoding (bytes) of one exact state given as 576 host bytes
    (bytes, bytearray or a uint8 numpy array / CPU tensor)."""
    import numpy as np
    a = np.ascontiguousarray(np.frombuffer(bytes(state), dtype=np.uint8)
                             if isinstance(state, (bytes, bytearray))
                             else np.asarray(state, dtype=np.uint8).reshape(-1))
    if a.size != STATE_BYTES:
        raise ValueError("a state is %d bytes" % STATE_BYTES)
    buf = ctypes.create_string_buffer(STATE_ENCODED_MAX)
    n = ctypes.c_size_t(0)
    _check(_lib.xsum_state_encode(a.ctypes.data, buf, STATE_ENCODED_MAX, ctypes.byref(n)))
    return buf.raw[:n.value]


def xsum_state_decode(data):
    """576-byte canonical state (bytes) from an encoding."""
    data = bytes(data)
    out = ctypes.create_string_buffer(STATE_BYTES)
    _check(_lib.xsum_state_decode(data, len(data), out))
    return out.raw


def xsum_segmented_plan(segs, out_dtype=SAME, tuning=None):
    """Plan for the segment descriptors `segs` (a numpy array with fields
    byte_offset u8, length u8, dtype u4, reserved u4, 24 bytes each, on the
    host).  Returns an opaque plan handle (int); free with xsum_plan_destroy."""
    import numpy as np
    a = np.ascontiguousarray(segs)
    if a.dtype.itemsize != 24:
        raise ValueError("segment descriptors must be 24-byte records")
    handle = ctypes.c_void_p()
    _check(_lib.xsum_segmented_plan(a.ctypes.data if a.size else None, a.size,
                                    out_dtype, ctypes.byref(tuning) if tuning else None,
                                    ctypes.byref(handle)))
    return handle.value


def xsum_plan_destroy(plan):
    _lib.xsum_plan_destroy(_p(plan))


def xsum_plan_get_info(plan):
    info = PlanInfo()
    _check(_lib.xsum_plan_get_info(_p(plan), ctypes.byref(info)))
    d = {k: getattr(info, k) for k, _ in PlanInfo._fields_ if k != "reserved"}
    d["lane_max"] = list(info.lane_max)
    d["wave_max"] = list(info.wave_max)
    return d


def xsum_plan_workspace_size(plan):
    return int(_lib.xsum_plan_workspace_size(_p(plan)))


def xsum_segmented_workspace_size(nseg, total_elems):
    return int(_lib.xsum_segmented_workspace_size(nseg, total_elems))


def xsum_exact_sum_segmented(base, segs, nseg, out_dtype, out, flags, ws, ws_bytes,
                             stream=0):
    """One-shot segmented sums; segs is a device or host address of nseg
    24-byte descriptors."""
    _check(_lib.xsum_exact_sum_segmented(_p(base), _p(segs), nseg, out_dtype, _p(out),
                                         _p(flags), _p(ws), ws_bytes, _p(stream)))


def xsum_segmented_workspace_init(ws, nbytes, stream=0):
    _check(_lib.xsum_segmented_workspace_init(_p(ws), nbytes, _p(stream)))


def xsum_segmented_run(plan, base, out, flags, ws, ws_bytes, stream=0):
    _check(_lib.xsum_segmented_run(_p(plan), _p(base), _p(out), _p(flags), _p(ws),
                                   ws_bytes, _p(stream)))


def xsum_segmented_run_noalloc(plan, base, out, flags, stream=0):
    _check(_lib.xsum_segmented_run_noalloc(_p(plan), _p(base), _p(out), _p(flags),
                                           _p(stream)))


def xsum_segmented_capture(plan, base, out, flags, ws, ws_bytes):
    g = ctypes.c_void_p()
    _check(_lib.xsum_segmented_capture(_p(plan), _p(base), _p(out), _p(flags), _p(ws),
                                       ws_bytes, ctypes.byref(g)))
    return g.value


def xsum_graph_launch(graph, stream=0):
    _check(_lib.xsum_graph_launch(_p(graph), _p(stream)))


def xsum_graph_destroy(graph):
    _lib.xsum_graph_destroy(_p(graph))


def xsum_batch_item_tasks(ptr, length, dtype, chunk_vectors):
    return int(_lib.xsum_batch_item_tasks(ptr, length, dtype, chunk_vectors))


def xsum_batch_add(items, nitems, ntasks, chunk_vectors, states, ctl, stream=0):
    _check(_lib.xsum_batch_add(_p(items), nitems, ntasks, chunk_vectors, _p(states),
                               _p(ctl), _p(stream)))


def xsum_batch_finalize(slots, fmts, n, states, out, flags, stream=0):
    _check(_lib.xsum_batch_finalize(_p(slots), _p(fmts), n, _p(states), _p(out),
                                    _p(flags), _p(stream)))


def xsum_probe_read(x, nbytes, sink, stream=0):
    """Measurement only: stream nbytes at x once (the binary64 kernel's
    access pattern, no arithmetic)."""
    _check(_lib.xsum_probe_read(_p(x), nbytes, _p(sink), _p(stream)))


def xsum_probe_flush(buf, nbytes, value=0, stream=0):
    """Measurement only: fill nbytes at buf with a 32-bit value."""
    _check(_lib.xsum_probe_flush(_p(buf), nbytes, value, _p(stream)))


def xsum_probe_clock(out, nsamples, interval_ticks, stream=0):
    """Measurement only: sample (100 MHz counter, shader clock counter)
    nsamples times, every interval_ticks ticks, into out[2i], out[2i+1]."""
    _check(_lib.xsum_probe_clock(_p(out), nsamples, interval_ticks, _p(stream)))


# ----------------------------------------------------- torch marshalling --

def xsum_truncated_workspace_size():
    return _lib.xsum_truncated_workspace_size()


def xsum_truncated_round(x, n, dtype, out_dtype, r, root, ws, ws_bytes, stream=0):
    """One Section 4 pass with truncation parameter r; writes the root record
    (TruncRoot layout) to device address root."""
    _check(_lib.xsum_truncated_round(_p(x), n, dtype, out_dtype, r, _p(root), _p(ws),
                                     ws_bytes, _p(stream)))


def xsum_exact_sum_truncated(x, n, dtype, out_dtype, ws, ws_bytes, stream=0):
    """Blocking Section 4 iteration.  Returns (result bit pattern, flags, r of
    the certifying pass or 0 for the untruncated one)."""
    out = ctypes.c_uint64(0)
    flags = ctypes.c_uint32(0)
    r = ctypes.c_int(-1)
    _check(_lib.xsum_exact_sum_truncated(_p(x), n, dtype, out_dtype, ctypes.byref(out),
                                         ctypes.byref(flags), ctypes.byref(r), _p(ws),
                                         ws_bytes, _p(stream)))
    ob = OUT_BYTES[(F64 if dtype == F64 else F32) if out_dtype == SAME else out_dtype]
    return out.value & ((1 << (8 * ob)) - 1), flags.value, r.value


def read_trunc_root(dev_tensor):
    """TruncRoot from the device bytes of a record (a uint8 CUDA tensor)."""
    raw = bytes(dev_tensor.cpu().numpy().tobytes())
    return TruncRoot.from_buffer_copy(raw[:ctypes.sizeof(TruncRoot)])


def stream_handle(stream=None):
    """Raw hipStream_t of a torch stream (default: the current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def dtype_of(tensor, dtype=None):
    """Library dtype code for a tensor: float64/float32/bfloat16 by type; raw
    bit-pattern tensors (integer types) need an explicit dtype."""
    import torch
    if dtype is not None:
        return dtype
    m = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
    if tensor.dtype not in m:
        raise ValueError("pass dtype= for a tensor of type %s" % tensor.dtype)
    return m[tensor.dtype]


def element_count(tensor, dtype):
    return tensor.numel() * tensor.element_size() // {F64: 8, F32: 4, BF16: 2}[dtype]


def exact_sum(tensor, dtype=None, out_dtype=SAME, stream=None):
    """Blocking exact sum of a contiguous device tensor.
    Returns (result bit pattern, flags)."""
    if not tensor.is_contiguous():
        raise ValueError("tensor must be contiguous")
    d = dtype_of(tensor, dtype)
    return xsum_exact_sum(tensor.data_ptr(), element_count(tensor, d), d,
                          out_dtype, stream_handle(stream))


class SegmentedSum:
    """A plan plus its device workspace, for repeated runs over one
    descriptor set.  base/out/flags are device tensors or raw pointers."""

    def __init__(self, segs, out_dtype=SAME, tuning=None, device="cuda", stream=None):
        import torch
        self.plan = xsum_segmented_plan(segs, out_dtype, tuning)
        self.nseg = len(segs)
        self.ws_bytes = max(8, xsum_plan_workspace_size(self.plan))
        self.workspace = torch.empty(self.ws_bytes // 8 + 1, dtype=torch.int64, device=device)
        xsum_segmented_workspace_init(self.workspace.data_ptr(), self.ws_bytes,
                                      stream_handle(stream))
        self.info = xsum_plan_get_info(self.plan)

    def run(self, base, out, flags=None, stream=None):
        p = lambda t: (t.data_ptr() if hasattr(t, "data_ptr") else int(t)) if t is not None else 0
        xsum_segmented_run(self.plan, p(base), p(out), p(flags), self.workspace.data_ptr(),
                           self.ws_bytes, stream_handle(stream))

    def capture(self, base, out, flags=None):
        p = lambda t: (t.data_ptr() if hasattr(t, "data_ptr") else int(t)) if t is not None else 0
        return xsum_segmented_capture(self.plan, p(base), p(out), p(flags),
                                      self.workspace.data_ptr(), self.ws_bytes)

    def close(self):
        if self.plan:
            xsum_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_states(count=1, device="cuda", stream=None):
    """count zeroed xsum_acc_t states in a device uint8 tensor [count, 576]."""
    import torch
    t = torch.empty((count, STATE_BYTES), dtype=torch.uint8, device=device)
    xsum_acc_zero(t.data_ptr(), count, stream_handle(stream))
    return t
