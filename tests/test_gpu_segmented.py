"""GPU parity of segmented sums (xsum_segmented_plan / run / capture): every
segment's result and flags equal the oracle's, for lane-group, whole-wave and
chunked segments, all formats, any tuning, and across graph replays."""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

NAMES = ["f64", "f32", "bf16"]
UINT = {0: np.uint64, 1: np.uint32, 2: np.uint16}
SIZE = {0: 8, 1: 4, 2: 2}


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401
    oracle.build_binned(force=False)


def expected(buf, desc, out_fmt=None):
    """Oracle (bits, flags) per segment."""
    want = oracle.segmented_oracle_sums(buf, desc["byte_offset"], desc["length"],
                                        desc["dtype"], out_fmt=out_fmt)
    return (np.array([w[0] for w in want], dtype=np.uint64),
            np.array([w[1] for w in want], dtype=np.uint32))


def run_gpu(buf, desc, out_mode=None, tuning=None, repeats=1):
    import torch
    import paper_1605_05436_amd as xs
    dbuf = torch.from_numpy(buf).to("cuda")
    om = xs.SAME if out_mode is None else {"f64": 0, "f32": 1, "bf16": 2}[out_mode]
    ss = xs.SegmentedSum(desc, om, tuning)
    out = torch.zeros(len(desc), dtype=torch.int64, device="cuda")
    fl = torch.zeros(len(desc), dtype=torch.int32, device="cuda")
    results = []
    for _ in range(repeats):
        out.fill_(-1)
        fl.fill_(-1)
        ss.run(dbuf, out, fl)
        torch.cuda.synchronize()
        results.append((out.cpu().numpy().view(np.uint64).copy(),
                        fl.cpu().numpy().view(np.uint32).copy()))
    info = ss.info
    ss.close()
    return results, info


def check(buf, desc, out_mode=None, tuning=None, repeats=1):
    want = expected(buf, desc, out_mode)
    results, info = run_gpu(buf, desc, out_mode, tuning, repeats)
    for got in results:
        bad = np.nonzero((got[0] != want[0]) | (got[1] != want[1]))[0]
        assert bad.size == 0, ("mismatching segments", bad[:10].tolist(),
                               desc[bad[:3]].tolist(), got[0][bad[:3]], want[0][bad[:3]])
    return info


def test_lognormal_batch_mixed_formats():
    buf, desc = workloads.config4(nseg=20_000, seed=1)
    info = check(buf, desc, repeats=2)
    assert info["wave_segments"] > 0 and info["lane_segments"] > 0


def test_edge_segments():
    rng = np.random.default_rng(3)
    lengths = [0, 1, 2, 3, 7, 8, 9, 63, 64, 65, 4095, 4096, 4097, 8191, 8193,
               16383, 16385, 100_000, 0, 1]
    dtypes = [int(rng.integers(0, 3)) for _ in lengths]
    buf, desc = workloads.config4(lengths=lengths, dtypes=dtypes, seed=4, kmin=-1000, kmax=1000,
                                  align=16)
    # misalign some starts by whole elements (offsets stay element-aligned)
    shift = np.array([SIZE[d] * (i % 3) for i, d in enumerate(dtypes)], dtype=np.uint64)
    nbuf = np.zeros(len(buf) + 64, dtype=np.uint8)
    for i in range(len(desc)):
        o, L, d = int(desc["byte_offset"][i]), int(desc["length"][i]), int(desc["dtype"][i])
        no = o + int(shift[i])
        nbuf[no:no + L * SIZE[d]] = buf[o:o + L * SIZE[d]]
        desc["byte_offset"][i] = no
    # specials in a few segments
    for i, pat in ((5, None), (13, None), (17, None)):
        o, d = int(desc["byte_offset"][i]), int(desc["dtype"][i])
        if int(desc["length"][i]) > 2:
            special = {0: 0x7FF0000000000000, 1: 0x7F800000, 2: 0x7F80}[d]
            nbuf[o:o + SIZE[d]] = np.array([special], dtype=UINT[d]).view(np.uint8)
    check(nbuf, desc)
    for om in ("f64", "f32", "bf16"):
        check(nbuf, desc, out_mode=om)


@pytest.mark.parametrize("lane_max,wave_max,chunk_vectors",
                         [(1, 1, 64), (100, 1000, 256), (1 << 20, 0, 0), (0, 0, 64 * 3 + 1),
                          (1, 1 << 40, 0), (50, 5000, 64 * 5 + 7)])
def test_tuning_does_not_change_bits(lane_max, wave_max, chunk_vectors):
    import paper_1605_05436_amd as xs
    buf, desc = workloads.config4(nseg=3000, seed=5, kmin=-300, kmax=300)
    t = xs.SegTuning()
    for d in range(3):
        t.lane_max[d] = lane_max
        t.wave_max[d] = wave_max
    t.chunk_vectors = chunk_vectors
    info = check(buf, desc, tuning=t)
    if lane_max == 1:
        assert info["lane_segments"] <= int((desc["length"] <= 1).sum())
    if wave_max == 1:
        assert info["wave_segments"] == 0 and info["chunked_segments"] > 0
    if wave_max == 1 << 40:
        assert info["chunked_segments"] == 0 and info["wave_segments"] > 0


def test_single_long_segment_equals_single_sum():
    bits = workloads.family("mixed", 3_000_001, 2000, seed=9)
    buf = bits.view(np.uint8)
    desc = np.zeros(1, dtype=workloads.SEGMENT_DTYPE)
    desc["length"] = len(bits)
    check(buf, desc)


def test_graph_replay_matches_eager():
    import torch
    import paper_1605_05436_amd as xs
    buf, desc = workloads.config4(nseg=5000, seed=6)
    want = expected(buf, desc)
    dbuf = torch.from_numpy(buf).to("cuda")
    ss = xs.SegmentedSum(desc)
    out = torch.zeros(len(desc), dtype=torch.int64, device="cuda")
    fl = torch.zeros(len(desc), dtype=torch.int32, device="cuda")
    graph = ss.capture(dbuf, out, fl)
    try:
        for rep in range(4):
            out.fill_(0)
            fl.fill_(0)
            xs.xsum_graph_launch(graph, xs.stream_handle())
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), want[0]), rep
            assert np.array_equal(fl.cpu().numpy().view(np.uint32), want[1]), rep
            # eager work between replays
            ss.run(dbuf, out, fl)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), want[0])
    finally:
        xs.xsum_graph_destroy(graph)
        ss.close()


def test_autotuner_picks_a_candidate_with_identical_results(tmp_path, monkeypatch):
    import torch
    import paper_1605_05436_amd as xs
    from paper_1605_05436_amd import autotune
    monkeypatch.setenv("XSUM_TUNE_CACHE", str(tmp_path / "tune.json"))
    buf, desc = workloads.config4(nseg=4000, seed=11)
    dbuf = torch.from_numpy(buf).to("cuda")
    cands = autotune.DEFAULT_CANDIDATES[:4]
    best, table = autotune.tune_segmented(desc, dbuf, candidates=cands, reps=2,
                                          per_bucket=True)
    # the global knobs come from one candidate; the per-bucket tables are the
    # tuner's own (the whole-batch comparison adds one table entry)
    assert best[:7] in [autotune._full(c)[:7] for c in cands]
    assert len(cands) <= len(table) <= len(cands) + 1
    # cached: the second call returns the same choice without timing
    best2, _ = autotune.tune_segmented(desc, dbuf, candidates=cands, reps=2)
    assert best2 == best
    want = expected(buf, desc)
    results, _ = run_gpu(buf, desc, tuning=autotune.tuning_struct(best))
    assert np.array_equal(results[0][0], want[0]) and np.array_equal(results[0][1], want[1])


def test_empty_plans_run_and_capture():
    """No segments, and only empty segments: runs and captured graphs work;
    an empty segment sums to +0."""
    import torch
    import paper_1605_05436_amd as xs
    dbuf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    empty = np.zeros(0, dtype=workloads.SEGMENT_DTYPE)
    ss = xs.SegmentedSum(empty)
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    ss.run(dbuf, out)
    g = ss.capture(dbuf, out)
    xs.xsum_graph_launch(g, xs.stream_handle())
    torch.cuda.synchronize()
    xs.xsum_graph_destroy(g)
    ss.close()
    zeros = np.zeros(300, dtype=workloads.SEGMENT_DTYPE)
    zeros["dtype"] = np.arange(300) % 3
    ss = xs.SegmentedSum(zeros)
    out = torch.full((300,), -1, dtype=torch.int64, device="cuda")
    fl = torch.full((300,), -1, dtype=torch.int32, device="cuda")
    g = ss.capture(dbuf, out, fl)
    for _ in range(3):
        out.fill_(-1)
        fl.fill_(-1)
        xs.xsum_graph_launch(g, xs.stream_handle())
        torch.cuda.synchronize()
        assert not out.cpu().numpy().any() and not fl.cpu().numpy().any()
    xs.xsum_graph_destroy(g)
    ss.close()


def test_all_chunked_plan_replays():
    """Every segment cut into chunks (per-segment states and tickets): three
    graph replays and an eager run in between give the oracle's bits each
    time, so the states and tickets return to zero after every launch."""
    import torch
    import paper_1605_05436_amd as xs
    buf, desc = workloads.config4(nseg=400, seed=8)
    want = expected(buf, desc)
    t = xs.SegTuning()
    for d in range(3):
        t.lane_max[d] = 1
        t.wave_max[d] = 1
    t.chunk_vectors = 64 * 3
    dbuf = torch.from_numpy(buf).to("cuda")
    ss = xs.SegmentedSum(desc, tuning=t)
    assert ss.info["chunked_segments"] == int((desc["length"] > 1).sum())
    out = torch.zeros(len(desc), dtype=torch.int64, device="cuda")
    fl = torch.zeros(len(desc), dtype=torch.int32, device="cuda")
    g = ss.capture(dbuf, out, fl)
    try:
        for rep in range(3):
            out.fill_(0)
            fl.fill_(0)
            xs.xsum_graph_launch(g, xs.stream_handle())
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), want[0]), rep
            assert np.array_equal(fl.cpu().numpy().view(np.uint32), want[1]), rep
            ss.run(dbuf, out, fl)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), want[0]), rep
    finally:
        xs.xsum_graph_destroy(g)
        ss.close()


def _oneshot(dbuf, desc, segs_on_device, ws, ws_bytes, out_mode=None):
    import torch
    import paper_1605_05436_amd as xs
    om = xs.SAME if out_mode is None else {"f64": 0, "f32": 1, "bf16": 2}[out_mode]
    out = torch.full((max(1, len(desc)),), -1, dtype=torch.int64, device="cuda")
    fl = torch.full((max(1, len(desc)),), -1, dtype=torch.int32, device="cuda")
    table = np.ascontiguousarray(desc)
    if segs_on_device:
        dsegs = torch.from_numpy(table.view(np.uint8).copy()).to("cuda")
        sp = dsegs.data_ptr()
    else:
        sp = table.ctypes.data
    xs.xsum_exact_sum_segmented(dbuf.data_ptr(), sp, len(desc), om, out.data_ptr(),
                                fl.data_ptr(), ws.data_ptr(), ws_bytes, xs.stream_handle())
    torch.cuda.synchronize()
    return (out.cpu().numpy().view(np.uint64)[:len(desc)],
            fl.cpu().numpy().view(np.uint32)[:len(desc)])


def test_oneshot_segmented_matches_oracle_in_a_bound_sized_workspace():
    # one-shot call: table on the device and on the host, chunked segments
    # included, twice in a row on one workspace (the second with a smaller
    # table), every segment against the oracle
    import torch
    import paper_1605_05436_amd as xs
    rng = np.random.default_rng(41)
    lengths = np.concatenate([workloads.segment_lengths(3000, seed=41),
                              [300_000, 700_001, 1, 0, 131_073]]).astype(np.int64)
    dtypes = np.concatenate([workloads.segment_dtypes(3000, seed=42),
                             [0, 0, 1, 2, 0]]).astype(np.int64)
    buf, desc = workloads.config4(nseg=len(lengths), seed=43, lengths=lengths,
                                  dtypes=dtypes)
    dbuf = torch.from_numpy(buf).to("cuda")
    total = int(desc["length"].sum())
    ws_bytes = xs.xsum_segmented_workspace_size(len(desc), total)
    ws = torch.empty(ws_bytes // 8 + 64, dtype=torch.int64, device="cuda")
    ws.fill_(-1)              # the call zeroes what must start at zero
    want = oracle.segmented_oracle_sums(buf, desc["byte_offset"], desc["length"],
                                        desc["dtype"])
    wb = np.array([w[0] for w in want], dtype=np.uint64)
    wf = np.array([w[1] for w in want], dtype=np.uint32)
    for on_dev in (True, False):
        got = _oneshot(dbuf, desc, on_dev, ws, ws_bytes)
        assert np.array_equal(got[0], wb) and np.array_equal(got[1], wf)
    sub = desc[::3].copy()
    got = _oneshot(dbuf, sub, True, ws, ws_bytes, out_mode="f32")
    want32 = oracle.segmented_oracle_sums(buf, sub["byte_offset"], sub["length"],
                                          sub["dtype"], out_fmt="f32")
    assert [(int(b), int(f)) for b, f in zip(*got)] == want32


def test_oneshot_segmented_rejects_a_small_workspace():
    import torch
    import paper_1605_05436_amd as xs
    buf, desc = workloads.config4(nseg=200, seed=44)
    dbuf = torch.from_numpy(buf).to("cuda")
    ws = torch.zeros(64, dtype=torch.int64, device="cuda")
    with pytest.raises(xs.XsumError) as e:
        _oneshot(dbuf, desc, False, ws, 512)
    assert e.value.status == xs.EINVAL and "workspace" in str(e.value)


def _tuned(lanes, unroll):
    import paper_1605_05436_amd as xs
    t = xs.SegTuning()
    for d in range(3):
        for b in range(xs.TUNE_BUCKETS):
            t.lanes[d][b] = lanes
            t.lane_unroll[d][b] = unroll
    return t


@pytest.mark.parametrize("kmin,kmax", [(-50, 50), (-1000, 1000)])
@pytest.mark.parametrize("lanes,unroll", [(1, 16), (2, 8), (4, 16), (8, 16), (8, 8),
                                          (16, 16), (16, 8)])
def test_lanes_per_segment_and_unroll_keep_the_bits(lanes, unroll, kmin, kmax):
    """Every lanes-per-segment and vectors-in-flight choice, on a narrow and
    a full-width exponent range (few or many active rows per lane)."""
    buf, desc = workloads.config4(nseg=2500, seed=21, kmin=kmin, kmax=kmax)
    check(buf, desc, tuning=_tuned(lanes, unroll))


def _patterned_segments(rng):
    """Segments whose active rows sit at the edges of the column: subnormals
    only (rows 0-1), +-DBL_MAX (the top rows), zeros mixed with one value,
    signed zeros, a special value, one tiny and one huge value together,
    and binary32 / bfloat16 at both ends of their ranges."""
    f64 = []
    sub = rng.integers(1, 1 << 52, size=700, dtype=np.uint64)
    sub |= rng.integers(0, 2, size=700, dtype=np.uint64) << np.uint64(63)
    f64.append(sub)
    big = np.full(301, 0x7FEFFFFFFFFFFFFF, dtype=np.uint64)
    big[::2] |= np.uint64(1 << 63)
    f64.append(big)
    z = np.zeros(999, dtype=np.uint64)
    z[500] = 0x3FF0000000000001
    f64.append(z)
    f64.append(np.full(64, 1 << 63, dtype=np.uint64))          # -0.0
    sp = workloads.config1(900, seed=7)
    sp[450] = 0x7FF0000000000000
    f64.append(sp)
    two = np.zeros(5000, dtype=np.uint64)
    two[0], two[4999] = 1, 0x7FE0000000000000
    f64.append(two)
    f32 = [np.full(333, 0x7F7FFFFF, dtype=np.uint32), np.arange(1, 800, dtype=np.uint32),
           np.zeros(257, dtype=np.uint32)]
    bf = [np.full(2049, 0x7F7F, dtype=np.uint16), np.arange(1, 3000, dtype=np.uint16) & 0x807F]
    return [(0, a) for a in f64] + [(1, a) for a in f32] + [(2, a) for a in bf]


@pytest.mark.parametrize("lanes", [0, 1, 4, 16])
def test_window_edges(lanes):
    rng = np.random.default_rng(22)
    specs = _patterned_segments(rng)
    chunks, rows, at = [], [], 0
    for d, a in specs:
        raw = a.view(np.uint8)
        rows.append((at, len(a), d, 0))
        chunks.append(raw)
        pad = (-raw.size) % 16
        chunks.append(np.zeros(pad, dtype=np.uint8))
        at += raw.size + pad
    buf = np.concatenate(chunks)
    desc = np.array(rows, dtype=workloads.SEGMENT_DTYPE)
    t = _tuned(lanes, 16) if lanes else None
    check(buf, desc, tuning=t)
    check(buf, desc, out_mode="f32", tuning=t)
