"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (the library's persistent default grid).

* n = 2^28 binary64, cancelling pairs + 1% perturbations: the GPU result
  equals the oracle's, and the oracle's exact total equals the closed form
  (the sum of the replaced pairs only).
* n = 2^31 binary64 (16 GiB), N(0,1) * 2^k with subnormals and balanced
  +-DBL_MAX: exact result; with unbalanced +-DBL_MAX the sum overflows, and
  the exported exact state still equals the oracle's integer.
* 10^6 segments of config 4 from one captured graph: sampled segments equal
  the oracle's; all 10^6 results are identical across replays and plans.
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
    st = xs.new_states(1)
    xs.xsum_acc_add(st.data_ptr(), x.data_ptr(), n, xs.F64, xs.stream_handle())
    torch.cuda.synchronize()
    raw = st.cpu().numpy().reshape(-1)
    digits = raw[:68 * 8].view(np.int64).tolist()
    assert sum(d << (32 * j) for j, d in enumerate(digits)) == acc.total
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
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([np.arange(0, nseg, 997),
                                    np.argsort(desc["length"])[-50:],
                                    rng.choice(nseg, 300, replace=False)]))
    print("checking", len(idx), "sampled segments against the oracle", flush=True)
    for i in idx.tolist():
        o, L, d = int(desc["byte_offset"][i]), int(desc["length"][i]), int(desc["dtype"][i])
        seg = buf[o:o + L * SIZE[d]].view(UINT[d])
        if L > 50_000:
            want = oracle.oracle_sum_binned(seg, NAMES[d], threads=8)
        else:
            want = oracle.oracle_sum(seg, NAMES[d])
        assert (int(res[i]), int(rfl[i])) == tuple(want), (i, L, NAMES[d])
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
