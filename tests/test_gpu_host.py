"""GPU parity of sums over host-resident inputs (xsum_exact_sum_host and
xsum_acc_add_host): the array is streamed through the device in chunks, and
the result must equal the oracle's and the device-resident sum of the same
data bit for bit, for any chunk size, format, pageable or pinned memory."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import gpu_sum

pytestmark = pytest.mark.gpu

CODE = {"f64": 0, "f32": 1, "bf16": 2}


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401
    oracle.build_binned(force=False)


def host_sum(bits, fmt, out_fmt=None, chunk_bytes=0):
    import paper_1605_05436_amd as xs
    oc = xs.SAME if out_fmt is None else CODE[out_fmt]
    return xs.xsum_exact_sum_host(bits.ctypes.data if len(bits) else 0, len(bits),
                                  CODE[fmt], oc, chunk_bytes)


@pytest.mark.parametrize("chunk_bytes", [0, 4096, 65552, 1 << 20])
def test_f64_any_chunk_size(chunk_bytes):
    print("host f64 n=3000003 chunk", chunk_bytes, flush=True)
    bits = workloads.family("mixed", 3_000_003, 2000, seed=21)
    want = oracle.oracle_sum_binned(bits, "f64", threads=4)
    assert host_sum(bits, "f64", chunk_bytes=chunk_bytes) == tuple(want)
    assert gpu_sum(bits, "f64") == tuple(want)


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_narrow_formats_with_specials(fmt):
    print("host", fmt, flush=True)
    rng = np.random.default_rng(5)
    n = 1_234_567
    bits = workloads.family("mixed", n, 100, seed=6, fmt=fmt)
    want = oracle.oracle_sum_binned(bits, fmt, threads=4)
    assert host_sum(bits, fmt, chunk_bytes=12288) == tuple(want)
    for out in ("f64", "f32", "bf16"):
        assert host_sum(bits, fmt, out, chunk_bytes=8192) == \
            tuple(oracle.oracle_sum_binned(bits, fmt, out, threads=4))
    # an infinity in the last chunk and a NaN in the first
    inf = {"f32": 0x7F800000, "bf16": 0x7F80}[fmt]
    b2 = bits.copy()
    b2[n - 3] = inf
    got = host_sum(b2, fmt, chunk_bytes=8192)
    assert got == tuple(oracle.oracle_sum_binned(b2, fmt, threads=4))
    assert got[1] & oracle.FLAG_INF
    b2[int(rng.integers(0, 1000))] = inf | (1 << ({"f32": 22, "bf16": 6}[fmt]))
    got = host_sum(b2, fmt, chunk_bytes=8192)
    assert got == tuple(oracle.oracle_sum_binned(b2, fmt, threads=4))
    assert got[1] & oracle.FLAG_NAN


def test_empty_and_tiny():
    assert host_sum(np.zeros(0, dtype=np.uint64), "f64") == (0, 0)
    for n in (1, 2, 3, 17):
        bits = workloads.family("mixed", n, 50, seed=n)
        assert host_sum(bits, "f64") == tuple(oracle.oracle_sum(bits, "f64"))


def test_pinned_tensor_and_state_accumulation():
    """Two host arrays (one pinned tensor, one pageable numpy array) and one
    device array added into one state equal the oracle of the concatenation."""
    import torch
    import paper_1605_05436_amd as xs
    a = workloads.family("positive", 2_000_001, 300, seed=31)
    b = workloads.family("mixed", 1_500_000, 300, seed=32)
    c = workloads.family("zero_sum", 1_000_000, 300, seed=33)
    pinned = torch.empty(len(a), dtype=torch.int64).pin_memory()
    pinned.numpy()[:] = a.view(np.int64)
    assert xs.exact_sum_host(pinned, xs.F64, chunk_bytes=1 << 20) == \
        tuple(oracle.oracle_sum_binned(a, "f64", threads=4))
    st = xs.new_states(1)
    sh = xs.stream_handle()
    xs.xsum_acc_add_host(st.data_ptr(), pinned.data_ptr(), len(a), xs.F64, 0, sh)
    xs.xsum_acc_add_host(st.data_ptr(), b.ctypes.data, len(b), xs.F64, 65536, sh)
    dc = torch.from_numpy(c.view(np.int64)).to("cuda")
    xs.xsum_acc_add(st.data_ptr(), dc.data_ptr(), len(c), xs.F64, sh)
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    xs.xsum_acc_finalize(st.data_ptr(), xs.F64, out.data_ptr(), fl.data_ptr(), sh)
    torch.cuda.synchronize()
    got = (int(out.cpu().numpy().view(np.uint64)[0]), int(fl.cpu()[0]))
    want = oracle.oracle_sum_binned(np.concatenate([a, b, c]), "f64", threads=4)
    assert got == tuple(want)


def test_one_gib_pinned_matches_device_sum():
    """2^27 doubles (1 GiB) from pinned memory in the default 64 MiB chunks:
    same bits as the device-resident sum."""
    import time
    import torch
    import paper_1605_05436_amd as xs
    n = 1 << 27
    print("host f64 n=2^27 pinned", flush=True)
    bits, _ = workloads.config2(log2n=27, seed=3)
    pinned = torch.empty(n, dtype=torch.int64).pin_memory()
    pinned.numpy()[:] = bits.view(np.int64)
    t0 = time.perf_counter()
    got = xs.exact_sum_host(pinned, xs.F64)
    dt = time.perf_counter() - t0
    print("host-streamed: %.1f ms, %.1f GB/s" % (dt * 1e3, n * 8 / dt / 1e9), flush=True)
    dev = torch.from_numpy(bits.view(np.int64)).to("cuda")
    assert got == xs.exact_sum(dev, xs.F64)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    assert got == tuple(oracle.finish(acc, "f64"))
