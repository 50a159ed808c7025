"""The C-ABI library loads on a machine without a GPU, exports every function
that include/xsum.h declares, and rejects bad arguments before touching the
device (no compute calls here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h)
           for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h")]
LIB = os.path.join(ROOT, "paper_1605_05436_amd", "libxsum.so")


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(xsum_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libxsum.so is not built; run __graft_entry__.build()")
    # as in the binding: torch's HIP runtime first, so the library binds to it
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("xsum_exact_sum", "xsum_exact_sum_async", "xsum_acc_add",
                 "xsum_acc_merge", "xsum_acc_finalize", "xsum_acc_zero",
                 "xsum_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_1605_05436_amd as xs
    assert sorted(xs.EXPORTED) == declared_functions()
    for n in declared_functions():
        assert callable(getattr(xs, n))


def test_struct_size_matches_header(lib):
    import paper_1605_05436_amd as xs
    assert xs.STATE_BYTES == 68 * 8 + 4 + 4 + 3 * 8


def _err(lib):
    lib.xsum_last_error.restype = ctypes.c_char_p
    return lib.xsum_last_error().decode()


def test_bad_dtype_is_rejected_on_the_host(lib):
    out = ctypes.c_uint64()
    lib.xsum_exact_sum.restype = ctypes.c_int
    st = lib.xsum_exact_sum(ctypes.c_void_p(4096), ctypes.c_uint64(10), 7, 255,
                            ctypes.byref(out), None, None)
    assert st == 2 and "dtype" in _err(lib)


def test_null_and_misaligned_inputs_are_rejected(lib):
    out = ctypes.c_uint64()
    lib.xsum_exact_sum.restype = ctypes.c_int
    st = lib.xsum_exact_sum(None, ctypes.c_uint64(10), 0, 255, ctypes.byref(out),
                            None, None)
    assert st == 1 and "NULL" in _err(lib)
    st = lib.xsum_exact_sum(ctypes.c_void_p(4100), ctypes.c_uint64(10), 0, 255,
                            ctypes.byref(out), None, None)
    assert st == 1 and "aligned" in _err(lib)
    st = lib.xsum_exact_sum(ctypes.c_void_p(4096), ctypes.c_uint64(10), 0, 255,
                            None, None, None)
    assert st == 1


def test_bad_output_dtype_and_null_state(lib):
    lib.xsum_exact_sum_async.restype = ctypes.c_int
    st = lib.xsum_exact_sum_async(ctypes.c_void_p(4096), ctypes.c_uint64(1), 0, 9,
                                  ctypes.c_void_p(8192), None, ctypes.c_void_p(16384),
                                  None)
    assert st == 2
    st = lib.xsum_exact_sum_async(ctypes.c_void_p(4096), ctypes.c_uint64(1), 0, 0,
                                  ctypes.c_void_p(8192), None, None, None)
    assert st == 1
    lib.xsum_acc_add.restype = ctypes.c_int
    assert lib.xsum_acc_add(None, ctypes.c_void_p(4096), ctypes.c_uint64(1), 0, None) == 1
    lib.xsum_acc_merge.restype = ctypes.c_int
    assert lib.xsum_acc_merge(None, None, None) == 1
    lib.xsum_acc_finalize.restype = ctypes.c_int
    assert lib.xsum_acc_finalize(ctypes.c_void_p(4096), 3, ctypes.c_void_p(8192),
                                 None, None) == 2
    lib.xsum_exact_sum_async_blocks.restype = ctypes.c_int
    st = lib.xsum_exact_sum_async_blocks(ctypes.c_void_p(4096), ctypes.c_uint64(1), 0, 0,
                                         ctypes.c_void_p(8192), None,
                                         ctypes.c_void_p(16384), -1, None)
    assert st == 1


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must not load a second HIP
    runtime (torch bundles its own libamdhip64)."""
    import subprocess
    import sys
    code = ("import paper_1605_05436_amd as xs, torch, ctypes; "
            "print(len(xs._hip_runtimes_loaded()))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_host_streaming_arguments_are_checked_on_the_host(lib):
    """xsum_exact_sum_host / xsum_acc_add_host reject bad arguments before
    any device work (the checks run with no GPU present)."""
    out = ctypes.c_uint64()
    f = lib.xsum_exact_sum_host
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    buf = (ctypes.c_double * 8)()
    p = ctypes.addressof(buf)
    assert f(p, 8, 7, 255, ctypes.addressof(out), None, 0, None) == 2       # input dtype
    assert f(p, 8, 0, 9, ctypes.addressof(out), None, 0, None) == 2         # output dtype
    assert f(None, 8, 0, 255, ctypes.addressof(out), None, 0, None) == 1    # NULL input
    assert f(p + 4, 8, 0, 255, ctypes.addressof(out), None, 0, None) == 1   # misaligned
    assert f(p, 8, 0, 255, None, None, 0, None) == 1                        # NULL out
    for bad in (16, 4096 + 8, 1 << 35):                                     # chunk size
        assert f(p, 8, 0, 255, ctypes.addressof(out), None, bad, None) == 5
        assert "chunk_bytes" in _err(lib)
    g = lib.xsum_acc_add_host
    g.restype = ctypes.c_int
    g.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                  ctypes.c_uint64, ctypes.c_void_p]
    assert g(None, p, 8, 0, 0, None) == 1                                   # NULL state
    assert g(ctypes.c_void_p(4096), p, 8, 3, 0, None) == 2                  # input dtype


def test_python_structs_match_the_header_layout(tmp_path):
    """The binding's ctypes/numpy mirrors of the public structs have the
    sizes and field offsets the C compiler gives the header's structs."""
    import shutil
    import subprocess
    import numpy as np
    import paper_1605_05436_amd as xs
    import workloads
    if shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "xsum.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu\n", sizeof(xsum_acc_t), sizeof(xsum_segment_t),
           sizeof(xsum_seg_tuning_t), sizeof(xsum_plan_info_t), sizeof(xsum_batch_item_t),
           offsetof(xsum_seg_tuning_t, two_lanes_from));
    printf("%zu %zu %zu\n", offsetof(xsum_seg_tuning_t, blocks_per_cu),
           offsetof(xsum_plan_info_t, workspace_bytes), offsetof(xsum_batch_item_t, first_task));
    return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True,
                          check=True).stdout.split("\n")[:2]
    acc, seg, tun, info, item, two = map(int, a.split())
    bpc, wsb, first = map(int, b.split())
    assert acc == xs.STATE_BYTES
    assert seg == workloads.SEGMENT_DTYPE.itemsize
    assert tun == ctypes.sizeof(xs.SegTuning) and two == xs.SegTuning.two_lanes_from.offset
    assert bpc == xs.SegTuning.blocks_per_cu.offset
    assert info == ctypes.sizeof(xs.PlanInfo) and wsb == xs.PlanInfo.workspace_bytes.offset
    dt = xs.batch_item_dtype()
    assert item == dt.itemsize and first == dt.fields["first_task"][1]
    assert isinstance(np.dtype(dt), np.dtype)


def test_oneshot_segmented_rejects_bad_arguments_on_the_host(lib):
    f = lib.xsum_exact_sum_segmented
    f.restype = ctypes.c_int
    vp = ctypes.c_void_p
    f.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    # nothing to do
    assert f(None, None, 0, 255, None, None, None, 0, None) == 0
    # NULL table, base, out or workspace
    assert f(4096, None, 3, 255, 4096, None, 4096, 1 << 20, None) == 1
    assert f(None, 4096, 3, 255, 4096, None, 4096, 1 << 20, None) == 1
    assert f(4096, 4096, 3, 255, None, None, 4096, 1 << 20, None) == 1
    assert f(4096, 4096, 3, 255, 4096, None, None, 1 << 20, None) == 1
    # base not 16-byte aligned, workspace not 256-byte aligned
    assert f(4104, 4096, 3, 255, 4096, None, 4096, 1 << 20, None) == 1
    assert f(4096, 4096, 3, 255, 4096, None, 4096 + 128, 1 << 20, None) == 1
    assert "aligned" in _err(lib)
    # too many segments
    assert f(4096, 4096, 1 << 31, 255, 4096, None, 4096, 1 << 20, None) == 5


def test_segmented_workspace_bound_grows_with_the_batch(lib):
    f = lib.xsum_segmented_workspace_size
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    base = f(0, 0)
    assert base >= 256 and base % 8 == 0
    # per segment: a 24-byte descriptor, a 32-byte item, a 16-byte lane entry
    assert f(1000, 0) >= base + 1000 * (24 + 32 + 16)
    # a 2^30-element segment may be cut into 1 MiB chunks with one state
    assert f(1, 1 << 30) >= f(1, 0) + 576 + 32 * ((1 << 30) >> 17)
    for nseg, total in [(10, 100), (10**6, 2 * 10**9), (5, 1 << 40)]:
        assert f(nseg, total) <= f(nseg + 1, total) <= f(nseg + 1, total + (1 << 20))
    assert f(1 << 31, 0) == 0 and f(1, 1 << 51) == 0


def test_truncated_pass_rejects_bad_arguments_on_the_host(lib):
    vp = ctypes.c_void_p
    ws = lib.xsum_truncated_workspace_size
    ws.restype = ctypes.c_size_t
    ws.argtypes = []
    nbytes = ws()
    # control word, 2048 block slots of 256 bytes, the record, an exact state
    assert nbytes == 256 + 2048 * 256 + 256 + 768
    f = lib.xsum_truncated_round
    f.restype = ctypes.c_int
    f.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp,
                  ctypes.c_size_t, vp]
    good = (4096, 8, 0, 255, 2, 8192, 1 << 20, nbytes, None)
    for r in (0, 1, 3, 8, 256):
        assert f(*good[:4], r, *good[5:]) == 1
    assert "r must be" in _err(lib)
    assert f(4096, 8, 7, 255, 2, 8192, 1 << 20, nbytes, None) == 2
    assert f(4096, 8, 0, 9, 2, 8192, 1 << 20, nbytes, None) == 2
    assert f(None, 8, 0, 255, 2, 8192, 1 << 20, nbytes, None) == 1
    assert f(4100, 8, 0, 255, 2, 8192, 1 << 20, nbytes, None) == 1
    assert f(4096, 8, 0, 255, 2, None, 1 << 20, nbytes, None) == 1
    assert f(4096, 8, 0, 255, 2, 8192, (1 << 20) + 64, nbytes, None) == 1
    assert f(4096, 8, 0, 255, 2, 8192, 1 << 20, nbytes - 8, None) == 1
    assert f(4096, (1 << 31) + 1, 0, 255, 2, 8192, 1 << 20, nbytes, None) == 5
    g = lib.xsum_exact_sum_truncated
    g.restype = ctypes.c_int
    g.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp,
                  ctypes.c_size_t, vp]
    assert g(4096, 8, 0, 255, None, None, None, 1 << 20, nbytes, None) == 1
    assert g(4096, 8, 0, 255, 8192, None, None, None, nbytes, None) == 1


def test_truncated_record_layout_matches_the_header(tmp_path):
    import shutil
    import subprocess
    import paper_1605_05436_amd as xs
    if shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    src = tmp_path / "trunc.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "xsum.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(xsum_trunc_root_t),
           offsetof(xsum_trunc_root_t, value), offsetof(xsum_trunc_root_t, count),
           offsetof(xsum_trunc_root_t, bound_value), offsetof(xsum_trunc_root_t, certified),
           offsetof(xsum_trunc_root_t, bits), offsetof(xsum_trunc_root_t, r));
    return 0;
}
''')
    exe = tmp_path / "trunc"
    subprocess.run(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.split()))
    T = xs.TruncRoot
    assert got == [ctypes.sizeof(T), T.value.offset, T.count.offset, T.bound_value.offset,
                   T.certified.offset, T.bits.offset, T.r.offset]


def test_measurement_probes_reject_bad_arguments_on_the_host(lib):
    lib.xsum_probe_clock.restype = ctypes.c_int
    lib.xsum_probe_clock.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_void_p]
    assert lib.xsum_probe_clock(None, 0, 1, None) == 0          # nothing to sample
    assert lib.xsum_probe_clock(None, 4, 100, None) == 1
    assert lib.xsum_probe_clock(4100, 4, 100, None) == 1        # not 8-byte aligned
    assert lib.xsum_probe_clock(4096, (1 << 20) + 1, 1, None) == 5
    assert lib.xsum_probe_clock(4096, 4, 0, None) == 5
    assert lib.xsum_probe_clock(4096, 200_000, 5001, None) == 5   # over 10 s
    assert "10 s" in _err(lib)
    lib.xsum_probe_read.restype = ctypes.c_int
    lib.xsum_probe_read.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                    ctypes.c_void_p]
    assert lib.xsum_probe_read(4096, 0, None, None) == 0
    assert lib.xsum_probe_read(4096, 24, 8192, None) == 1        # not a multiple of 16
    lib.xsum_probe_flush.restype = ctypes.c_int
    lib.xsum_probe_flush.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_void_p]
    assert lib.xsum_probe_flush(4098, 8, 0, None) == 1
