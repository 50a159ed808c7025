"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (the library's persistent default grid).

* n = 2^28 binary64, cancelling pairs + 1% perturbations: the GPU result
  equals the oracle's, and the oracle's exact total equals the closed form
  (the sum of the replaced pairs only).
* n = 2^31 binary64 (16 GiB), N(0,1) * 2^k with subnormals and balanced
  +-DBL_MAX: exact result; with unbalanced +-DBL_MAX the sum overflows, and
  the exported exact state still equals the oracle's integer.
* 2^29 binary32 (cancelling pairs + perturbations) and 2^30 bfloat16 (mixed
  signs), 2 GiB each as the benchmark's narrow-format lines time them: the
  bfloat16 sum runs the 32-bit column entries with their periodic flushes.
* 10^6 segments of config 4 from one captured graph: every segment equals
  the oracle's; all 10^6 results are identical across replays and plans.
* Section 4's truncated iteration on the 2^28 and 2^31 binary64 inputs and
  the 2 GiB binary32 and bfloat16 ones: the same bits and flags as the
  oracle, and every pass (r = 2, 4, 16) within its bound of the oracle's
  exact integer.
"""

import gc

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import gpu_sum_async

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401
    oracle.build_binned(force=False)


def _device(bits):
    import torch
    return torch.from_numpy(bits.view(np.int64)).to("cuda")


def _release():
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def _check_truncated(x, n, acc, want, fmt="f64"):
    """Section 4's iteration equals the exact rounding; every pass's root is
    within its bound of the exact integer, and a certified pass carries the
    exact rounding."""
    import torch
    import paper_1605_05436_amd as xs
    code = {"f64": xs.F64, "f32": xs.F32, "bf16": xs.BF16}[fmt]
    wsb = xs.xsum_truncated_workspace_size()
    ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")
    got = xs.xsum_exact_sum_truncated(x.data_ptr(), n, code, xs.SAME, ws.data_ptr(), wsb,
                                      xs.stream_handle())
    assert got[:2] == want and got[2] in (2, 4, 16, 0)
    rec = torch.zeros(256, dtype=torch.uint8, device="cuda")
    for r in (2, 4, 16):
        print("truncated pass r=%d n=%d" % (r, n), flush=True)
        xs.xsum_truncated_round(x.data_ptr(), n, code, xs.SAME, r, rec.data_ptr(),
                                ws.data_ptr(), wsb, xs.stream_handle())
        torch.cuda.synchronize()
        root = xs.read_trunc_root(rec)
        s = sum(root.value[j] << (32 * root.index[j]) for j in range(root.count))
        bound = root.bound_value << (32 * root.bound_index) if root.bound_value else 0
        assert root.count <= r
        if not root.special:
            assert abs(acc.total - s) <= bound
        if root.certified:
            assert (root.bits, root.flags) == want


@pytest.mark.parametrize("variant", ["a", "b"])
def test_config2_full_size(variant):
    print("config2 variant", variant, "n=2^28", flush=True)
    bits, terms = workloads.config2(log2n=28, seed=0, variant=variant)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    assert acc.total == oracle.exact_sum_binned(terms, "f64")[0].total
    x = _device(bits)
    got = gpu_sum_async(x, len(bits), "f64")
    assert got[:2] == tuple(oracle.finish(acc, "f64"))
    assert got[2] == bytes(576)
    _check_truncated(x, len(bits), acc, tuple(oracle.finish(acc, "f64")))
    del x
    _release()


def test_config3_full_size_balanced():
    n = 1 << 31
    print("config3 balanced n=2^31", flush=True)
    bits = workloads.config3(n=n, seed=0)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    x = _device(bits)
    del bits
    got = gpu_sum_async(x, n, "f64")
    assert got[:2] == tuple(oracle.finish(acc, "f64"))
    _check_truncated(x, n, acc, tuple(oracle.finish(acc, "f64")))
    del x
    _release()


def test_config3_full_size_overflow_state():
    import torch
    import paper_1605_05436_amd as xs
    n = 1 << 31
    print("config3 unbalanced n=2^31", flush=True)
    bits = workloads.config3(n=n, seed=0, balanced=False)
    acc, _ = oracle.exact_sum_binned(bits, "f64")
    x = _device(bits)
    del bits
    got = gpu_sum_async(x, n, "f64")
    want = tuple(oracle.finish(acc, "f64"))
    assert got[:2] == want
    assert want[1] & oracle.FLAG_OVERFLOW
    _check_truncated(x, n, acc, want)
    st = xs.new_states(1)
    xs.xsum_acc_add(st.data_ptr(), x.data_ptr(), n, xs.F64, xs.stream_handle())
    torch.cuda.synchronize()
    raw = st.cpu().numpy().reshape(-1)
    digits = raw[:68 * 8].view(np.int64).tolist()
    assert sum(d << (32 * j) for j, d in enumerate(digits)) == acc.total
    del x
    _release()


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_narrow_formats_full_size(fmt):
    import torch
    n = (1 << 31) // {"f32": 4, "bf16": 2}[fmt]
    print("narrow format", fmt, "n =", n, flush=True)
    if fmt == "f32":
        bits = workloads.serving_payload(n, "f32", seed=0)
    else:
        piece = 1 << 26
        bits = np.concatenate([workloads.family("mixed", piece, 100, seed=i, fmt="bf16")
                               for i in range(n // piece)])
    acc, _ = oracle.exact_sum_binned(bits, fmt)
    x = torch.from_numpy(bits.view({"f32": np.int32, "bf16": np.int16}[fmt])).to("cuda")
    del bits
    want = tuple(oracle.finish(acc, "f32"))
    got = gpu_sum_async(x, n, fmt)
    assert got[:2] == want
    assert got[2] == bytes(576)
    # the same 2 GiB through a grid of 3 blocks: each wave carries ~170x more
    # tiles (bfloat16: hundreds of flushes of its 32-bit entries)
    got = gpu_sum_async(x, n, fmt, blocks=3)
    assert got[:2] == want
    assert got[2] == bytes(576)
    _check_truncated(x, n, acc, want, fmt)
    del x
    _release()


SIZE = {0: 8, 1: 4, 2: 2}
UINT = {0: np.uint64, 1: np.uint32, 2: np.uint16}
NAMES = ["f64", "f32", "bf16"]


def test_config4_full_size():
    """10^6 segments (lognormal lengths, three formats, 10.9 GB) replayed from
    one captured graph with the default plan, as the benchmark runs it:
    sampled segments equal the oracle's one by one; every segment's bits are
    the same on a second replay and under a plan that cuts the work
    differently (more whole-wave items and many chunked segments)."""
    import torch
    import paper_1605_05436_amd as xs
    print("config4 full size: 1e6 segments", flush=True)
    buf, desc = workloads.config4(nseg=1_000_000, seed=0)
    dbuf = torch.from_numpy(buf).to("cuda")
    nseg = len(desc)
    out = torch.zeros(nseg, dtype=torch.int64, device="cuda")
    fl = torch.zeros(nseg, dtype=torch.int32, device="cuda")
    ss = xs.SegmentedSum(desc)
    graph = ss.capture(dbuf, out, fl)
    results = []
    try:
        for _ in range(2):
            out.fill_(-1)
            fl.fill_(-1)
            xs.xsum_graph_launch(graph, xs.stream_handle())
            torch.cuda.synchronize()
            results.append((out.cpu().numpy().view(np.uint64).copy(),
                            fl.cpu().numpy().view(np.uint32).copy()))
    finally:
        xs.xsum_graph_destroy(graph)
        ss.close()
    assert np.array_equal(results[0][0], results[1][0])
    assert np.array_equal(results[0][1], results[1][1])
    res, rfl = results[0]
    print("checking all", nseg, "segments against the oracle", flush=True)
    want = oracle.segmented_oracle_sums(buf, desc["byte_offset"], desc["length"],
                                        desc["dtype"])
    wb = np.array([w[0] for w in want], dtype=np.uint64)
    wf = np.array([w[1] for w in want], dtype=np.uint32)
    bad = np.nonzero((wb != res) | (wf != rfl))[0]
    assert bad.size == 0, (bad[:10].tolist(), desc[bad[:3]].tolist())
    # a different cut of the same work
    t = xs.SegTuning()
    for d, (lm, wm) in enumerate(((1024, 1 << 16), (2048, 1 << 17), (4096, 1 << 18))):
        t.lane_max[d] = lm
        t.wave_max[d] = wm
    t.chunk_vectors = 1 << 14
    ss2 = xs.SegmentedSum(desc, tuning=t)
    assert ss2.info["chunked_segments"] > 1000
    out.fill_(-1)
    fl.fill_(-1)
    ss2.run(dbuf, out, fl)
    torch.cuda.synchronize()
    ss2.close()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), res)
    assert np.array_equal(fl.cpu().numpy().view(np.uint32), rfl)
    del dbuf, out, fl
    _release()
