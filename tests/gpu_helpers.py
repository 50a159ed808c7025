"""Helpers for the GPU parity tests: move bit-pattern arrays to the device and
call the library through its C-ABI binding."""

import numpy as np

FMT_CODE = {"f64": 0, "f32": 1, "bf16": 2}
SIGNED_VIEW = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32,
               np.dtype(np.uint16): np.int16}


def to_device(bits, offset_elems=0):
    """Device tensor holding bits; with offset_elems > 0 the data starts that
    many elements into a larger allocation (misaligned start)."""
    import torch
    sv = SIGNED_VIEW[bits.dtype]
    host = np.zeros(len(bits) + offset_elems, dtype=bits.dtype)
    host[offset_elems:] = bits
    t = torch.from_numpy(host.view(sv)).to("cuda")
    return t[offset_elems:]


def gpu_sum(bits, fmt, out_fmt=None, offset_elems=0):
    """Blocking library sum of the bit patterns; returns (bits, flags)."""
    import paper_1605_05436_amd as xs
    t = to_device(bits, offset_elems)
    out = xs.SAME if out_fmt is None else FMT_CODE[out_fmt]
    return xs.xsum_exact_sum(t.data_ptr() if len(bits) else 0, len(bits),
                             FMT_CODE[fmt], out, xs.stream_handle())


def gpu_sum_async(t, n, fmt, out_fmt=None, blocks=0, scratch=None):
    """Asynchronous library sum of a device tensor; returns (bits, flags,
    scratch state after the call as bytes)."""
    import torch
    import paper_1605_05436_amd as xs
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = xs.new_states(1) if scratch is None else scratch
    oc = xs.SAME if out_fmt is None else FMT_CODE[out_fmt]
    xs.xsum_exact_sum_async_blocks(t.data_ptr() if n else 0, n, FMT_CODE[fmt], oc,
                                   out.data_ptr(), flags.data_ptr(),
                                   st.data_ptr(), blocks, xs.stream_handle())
    torch.cuda.synchronize()
    of = oc if oc != xs.SAME else (0 if fmt == "f64" else 1)
    ob = xs.OUT_BYTES[of]
    val = int(out.cpu().numpy().view(np.uint64)[0]) & ((1 << (8 * ob)) - 1)
    return val, int(flags.cpu()[0]), st.cpu().numpy().tobytes()
