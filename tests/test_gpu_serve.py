"""GPU tests of the continuous-batching server: every result equals the
oracle, and a request's result is bit-identical whether it runs alone or in a
mix with others (tolerance: zero ulps), also under admission back-pressure."""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

FMTS = ["f64", "f32", "bf16"]
UINT = {"f64": np.uint64, "f32": np.uint32, "bf16": np.uint16}
SINT = {"f64": np.int64, "f32": np.int32, "bf16": np.int16}


@pytest.fixture(scope="module")
def pools():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401
    oracle.build_binned(force=False)
    host = {"f64": workloads.serving_payload(4_000_000, "f64", seed=1),
            "f32": workloads.serving_payload(4_000_000, "f32", seed=2)}
    host["bf16"] = (host["f32"] >> np.uint32(16)).astype(np.uint16)
    dev = {k: torch.from_numpy(v.view(SINT[k])).to("cuda") for k, v in host.items()}
    torch.cuda.synchronize()
    return host, dev


def make_requests(pools, count, seed, smax=3_000_000):
    from paper_1605_05436_amd.serve import Request
    host, dev = pools
    rng = np.random.default_rng(seed)
    reqs, want = [], []
    for i in range(count):
        fmt = FMTS[int(rng.integers(0, 3))]
        n = int(np.exp(rng.uniform(np.log(1), np.log(smax))))
        off = int(rng.integers(0, len(host[fmt]) - n + 1))
        reqs.append(Request(rid=i, src=dev[fmt][off:off + n], n=n,
                            dtype={"f64": 0, "f32": 1, "bf16": 2}[fmt]))
        want.append(tuple(oracle.oracle_sum_binned(host[fmt][off:off + n], fmt)))
    return reqs, want


def clone(r):
    from paper_1605_05436_amd.serve import Request
    return Request(rid=r.rid, src=r.src, n=r.n, dtype=r.dtype, out_dtype=r.out_dtype,
                   arrival=r.arrival)


def server(**kw):
    from paper_1605_05436_amd.serve import ExactSumServer
    args = dict(arena_bytes=256 << 20, slots=64, piece_elems=1 << 20,
                batch_bytes=16 << 20, chunk_vectors=4096, max_items=512, ring=4)
    args.update(kw)
    return ExactSumServer(**args)


def test_alone_and_in_the_mix_are_identical(pools):
    from paper_1605_05436_amd.serve import run_trace
    reqs, want = make_requests(pools, 40, seed=7)
    srv = server()
    alone = {}
    for r in reqs:
        done = run_trace(srv, [clone(r)], realtime=False)
        alone[r.rid] = (done[-1].bits, done[-1].flags)
    srv2 = server()
    mixed = run_trace(srv2, [clone(r) for r in reqs], realtime=False)
    assert len(mixed) == len(reqs)
    got = {r.rid: (r.bits, r.flags) for r in mixed}
    for r, w in zip(reqs, want):
        assert alone[r.rid] == w, r.rid
        assert got[r.rid] == w, r.rid
    assert srv2.batches < len(reqs)          # requests really shared batches


def test_backpressure_small_arena_and_few_slots(pools):
    from paper_1605_05436_amd.serve import run_trace
    reqs, want = make_requests(pools, 30, seed=8, smax=1_000_000)
    srv = server(arena_bytes=12 << 20, slots=3, batch_bytes=2 << 20, piece_elems=1 << 18)
    done = run_trace(srv, [clone(r) for r in reqs], realtime=False)
    got = {r.rid: (r.bits, r.flags) for r in done}
    assert [got[r.rid] for r in reqs] == want
    assert srv.alloc.free == [(0, 12 << 20)] and sorted(srv.free_slots) == [0, 1, 2]


def test_oversized_request_is_refused(pools):
    from paper_1605_05436_amd.serve import Request
    host, dev = pools
    srv = server(arena_bytes=1 << 20)
    with pytest.raises(ValueError):
        srv.submit(Request(rid=0, src=dev["f64"], n=len(host["f64"]), dtype=0))


def test_short_poisson_trace(pools):
    from paper_1605_05436_amd.serve import run_trace, latency_stats
    host, dev = pools
    t, size, dt = workloads.serving_trace(seed=3, rate=2000.0, duration=0.25, smin=1e3, smax=1e6)
    reqs, want = make_requests(pools, len(t), seed=9, smax=1_000_000)
    for r, a in zip(reqs, t):
        r.arrival = float(a)
    srv = server(arena_bytes=512 << 20, slots=256)
    done = run_trace(srv, reqs, realtime=True)
    assert len(done) == len(reqs)
    got = {r.rid: (r.bits, r.flags) for r in done}
    assert [got[r.rid] for r in reqs] == want
    st = latency_stats(done)
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"]
