"""Autotuner for segmented sums and the single-sum grid.

For a batch of segments the tunables decide which path each length bucket
takes and how work is cut.  Global knobs: lane_max (per-lane groups below
it), wave_max (one wave per segment below it), chunk_vectors (chunk size
above it), blocks_per_cu (resident one-wave groups per CU) and lane_buckets
(length buckets per doubling inside the per-lane path).  Per format and per
log2-size bucket of the lane-group segments: the lanes each segment gets (1
to 16) and the vectors each lane keeps in flight (8 or 16), which select
different kernel code for that bucket's work items.

The tuner first picks the global knobs by timing whole-batch candidate plans,
then, bucket by bucket, times each lanes/unroll choice on a plan of that
bucket's segments alone, and finally keeps the combined per-bucket table if
the whole batch runs faster with it.  Every candidate's results must be bit
identical to the first one's (exactness makes that a hard requirement, not a
tolerance).  Timings start after a warm-up long enough for the device clock
to settle, and candidates are timed in interleaved rounds (median per
candidate), so slow phases of the clock hit all of them alike.  Results are
cached in a JSON file keyed by the device architecture and a coarse
signature of the batch (per-format log2-length histogram), so later plans of
similar batches reuse them.

The cache path is $XSUM_TUNE_CACHE, else ~/.cache/xsum/tune.json.
"""

import hashlib
import json
import os
import time

import numpy as np

from . import (SegTuning, SegmentedSum, TUNE_BUCKETS, xsum_graph_launch,
               xsum_graph_destroy, stream_handle)

DEFAULT_CANDIDATES = [
    # (lane_max per dtype, wave_max per dtype, chunk_vectors, blocks_per_cu,
    #  lane_buckets, two_lanes_from, four_lanes_from); 0 = library default
    ((0, 0, 0), (0, 0, 0), 0, 0, 0, 0, 0),                  # library defaults
    ((8192, 8192, 16384), (0, 0, 0), 0, 0, 0, 0, 0),        # half the lane limits
    ((32768, 32768, 65536), (0, 0, 0), 0, 0, 0, 0, 0),      # twice them
    ((0, 0, 0), (0, 0, 0), 0, 0, 2, 0, 0),
    ((0, 0, 0), (0, 0, 0), 0, 0, 8, 0, 0),
    ((0, 0, 0), (1 << 16, 1 << 19, 1 << 20), 1 << 15, 0, 0, 0, 0),
    ((0, 0, 0), (1 << 19, 1 << 21, 1 << 22), 1 << 18, 0, 0, 0, 0),
    ((0, 0, 0), (0, 0, 0), 0, 3, 0, 0, 0),
    ((0, 0, 0), (0, 0, 0), 0, 0, 0, 1024, 8192),
    ((0, 0, 0), (0, 0, 0), 0, 0, 0, 4096, 1 << 40),
]


def cache_path():
    p = os.environ.get("XSUM_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "xsum", "tune.json")


def _arch():
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def batch_signature(desc):
    """Coarse signature of a batch: per-format histogram of log2 lengths,
    rounded to 5% of segments, plus the segment count's order of magnitude."""
    L = np.asarray(desc["length"], dtype=np.int64)
    D = np.asarray(desc["dtype"], dtype=np.int64)
    n = max(1, len(L))
    lg = np.where(L > 0, np.floor(np.log2(np.maximum(L, 1))), -1).astype(np.int64)
    hist = np.zeros((3, 23), dtype=np.int64)
    np.add.at(hist, (D, np.clip(lg + 1, 0, 22)), 1)
    q = np.round(hist * 20 / n).astype(np.int64)
    key = "%s|%d|%s" % (_arch(), int(np.log10(n)), q.tobytes().hex())
    return hashlib.sha1(key.encode()).hexdigest()[:16]


NB = TUNE_BUCKETS
EMPTY_TABLE = tuple(tuple(0 for _ in range(NB)) for _ in range(3))


def _tuning(c):
    """SegTuning from a candidate tuple (lane_max, wave_max, chunk_vectors,
    blocks_per_cu, lane_buckets[, two_lanes_from, four_lanes_from[, lanes,
    lane_unroll]]), the last two 3 x 24 tables."""
    lane, wave, chunk, bpc, buckets = c[:5]
    two, four = c[5:7] if len(c) >= 7 else (0, 0)
    lanes, unroll = c[7:9] if len(c) >= 9 else (EMPTY_TABLE, EMPTY_TABLE)
    t = SegTuning()
    for d in range(3):
        t.lane_max[d] = lane[d]
        t.wave_max[d] = wave[d]
        for b in range(NB):
            t.lanes[d][b] = lanes[d][b]
            t.lane_unroll[d][b] = unroll[d][b]
    t.chunk_vectors = chunk
    t.blocks_per_cu = bpc
    t.lane_buckets = buckets
    t.two_lanes_from = two
    t.four_lanes_from = four
    return t


def _full(c):
    """The candidate with all nine fields."""
    c = tuple(c)
    if len(c) < 7:
        c = c + (0, 0)
    if len(c) < 9:
        c = c + (EMPTY_TABLE, EMPTY_TABLE)
    return c


def _as_list(c):
    c = _full(c)
    return [list(c[0]), list(c[1])] + list(c[2:7]) + \
        [[list(r) for r in c[7]], [list(r) for r in c[8]]]


def _from_list(c):
    c = list(c)
    if len(c) >= 9:
        return (tuple(c[0]), tuple(c[1])) + tuple(c[2:7]) + \
            (tuple(tuple(r) for r in c[7]), tuple(tuple(r) for r in c[8]))
    return (tuple(c[0]), tuple(c[1])) + tuple(c[2:])


class _Graph:
    """One candidate plan captured for a batch, with its own outputs."""

    def __init__(self, desc, dbuf, cand):
        import torch
        self.ss = SegmentedSum(desc, tuning=_tuning(cand))
        n = max(1, len(desc))
        self.out = torch.zeros(n, dtype=torch.int64, device="cuda")
        self.flags = torch.zeros(n, dtype=torch.int32, device="cuda")
        self.g = self.ss.capture(dbuf, self.out, self.flags)

    def time(self, reps):
        import torch
        sh = stream_handle()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        xsum_graph_launch(self.g, sh)
        e0.record()
        for _ in range(reps):
            xsum_graph_launch(self.g, sh)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def results(self):
        return self.out.cpu().numpy().copy(), self.flags.cpu().numpy().copy()

    def close(self):
        xsum_graph_destroy(self.g)
        self.ss.close()


def warm_up(graph, ms=150.0):
    """Replay a graph for about `ms` milliseconds: the device clock drops
    when a sustained load starts and takes tens of milliseconds to settle."""
    import torch
    t0 = time.time()
    while (time.time() - t0) * 1e3 < ms:
        graph.time(4)
    torch.cuda.synchronize()


def _time_interleaved(desc, dbuf, cands, reps, rounds, verbose=False, tag=""):
    """Capture every candidate, time them round-robin `rounds` times (reps
    replays each), return [(cand, median ms)] and check that all results are
    bit-identical to the first candidate's."""
    graphs = [_Graph(desc, dbuf, c) for c in cands]
    try:
        warm_up(graphs[0])
        times = [[] for _ in cands]
        for _ in range(rounds):
            for i, g in enumerate(graphs):
                times[i].append(g.time(reps))
        ref = graphs[0].results()
        for c, g in zip(cands, graphs):
            res = g.results()
            if not (np.array_equal(res[0], ref[0]) and np.array_equal(res[1], ref[1])):
                raise RuntimeError("autotune candidate %r changed the results" % (c,))
    finally:
        for g in graphs:
            g.close()
    table = [(c, float(np.median(t))) for c, t in zip(cands, times)]
    if verbose:
        for c, m in table:
            print("[autotune]%s %r: %.4f ms" % (tag, c if len(str(c)) < 200 else "...", m),
                  flush=True)
    return table


def _pick(table, margin):
    """First entry unless another is faster by more than margin."""
    best = table[0]
    for c, m in table[1:]:
        if m < best[1] * (1.0 - margin):
            best = (c, m)
    return best


LANE_CHOICES = (1, 2, 4, 8, 16)


def default_lanes(nbytes, two_from=2048, four_from=32768):
    """Lanes per segment the planner gives a lane-group segment of nbytes
    bytes when the tuning table leaves its bucket at 0."""
    return 1 if nbytes < two_from else 2 if nbytes < four_from else 4


def lane_buckets_of(desc, lane_max):
    """(format, size bucket) -> indices of the segments that lane groups sum
    (length <= lane_max of the format), bucket = floor(log2 bytes)."""
    L = np.asarray(desc["length"], dtype=np.int64)
    D = np.asarray(desc["dtype"], dtype=np.int64)
    es = np.array([8, 4, 2], dtype=np.int64)[D]
    lm = np.array(lane_max, dtype=np.int64)[D]
    nb = L * es
    b = np.where(nb > 0, np.floor(np.log2(np.maximum(nb, 1))), 0).astype(np.int64)
    b = np.minimum(b, NB - 1)
    groups = {}
    sel = np.nonzero(L <= lm)[0]
    for d in range(3):
        for bb in range(NB):
            idx = sel[(D[sel] == d) & (b[sel] == bb)]
            if len(idx):
                groups[(d, bb)] = idx
    return groups


def tune_buckets(desc, dbuf, base, reps=6, rounds=3, min_frac=0.01, margin=0.01,
                 verbose=False):
    """Lanes per segment for each (format, size bucket) of lane-group
    segments, chosen in the context of the batch: buckets are visited
    largest first, and each one's choices are timed on the whole share of
    its format (the other buckets as chosen so far), since a bucket timed
    alone is dominated by the launch's fixed costs.  Buckets holding less
    than min_frac of their format's bytes keep the planner's choice.
    Returns (lanes table, unroll table, per-bucket timings)."""
    base = _full(base)
    lane_max = [v or dflt for v, dflt in zip(base[0], (16384, 16384, 32768))]
    two = base[5] or 2048
    four = base[6] or 32768
    es = [8, 4, 2]
    L = np.asarray(desc["length"], dtype=np.int64)
    D = np.asarray(desc["dtype"], dtype=np.int64)
    lanes = [[0] * NB for _ in range(3)]
    unroll = [list(r) for r in base[8]]
    for d in range(3):
        for b in range(NB):
            lanes[d][b] = base[7][d][b] or default_lanes(1 << b, two, four)
    detail = {}
    groups = lane_buckets_of(desc, lane_max)
    for d in range(3):
        share = np.ascontiguousarray(desc[D == d])
        total = int(L[D == d].sum()) * es[d]
        if len(share) == 0 or total == 0:
            continue
        order = sorted(((int(L[idx].sum()) * es[d], b) for (dd, b), idx in groups.items()
                        if dd == d), reverse=True)
        for nbytes, b in order:
            if nbytes < min_frac * total:
                continue
            cur = lanes[d][b]
            choices = [cur] + [g for g in LANE_CHOICES if g != cur]
            cands = []
            for g in choices:
                tl = [list(r) for r in lanes]
                tl[d][b] = g
                cands.append(base[:7] + (tuple(map(tuple, tl)), tuple(map(tuple, unroll))))
            table = _time_interleaved(share, dbuf, cands, reps, rounds)
            best = _pick(table, margin)[0]
            lanes[d][b] = best[7][d][b]
            detail["%d/%d" % (d, b)] = [[g, round(m, 5)] for g, (_, m) in zip(choices, table)]
            if verbose:
                print("[autotune] format %d bucket 2^%d (%.1f MB): %s -> %d lanes"
                      % (d, b, nbytes / 1e6, " ".join("%d:%.4f" % (g, m) for g, (_, m)
                                                      in zip(choices, table)),
                         lanes[d][b]), flush=True)
    return lanes, unroll, detail


def tune_segmented(desc, dbuf, candidates=None, reps=4, rounds=3, use_cache=True,
                   verbose=False, margin=0.03, per_bucket=True):
    """Pick the fastest tuning for this batch.  Returns (tuning tuple, table)
    where table lists (candidate, ms) of the global stage plus, with
    per_bucket, the per-bucket table candidate.  Raises if candidates
    disagree.  The first candidate (the library defaults) is kept unless
    another is faster by more than `margin` (relative), so near-ties between
    timings resolve the same way from run to run."""
    sig = batch_signature(desc)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if sig in cache:
            return _from_list(cache[sig]["tuning"]), cache[sig]["table"]
    cands = [_full(c) for c in (candidates or DEFAULT_CANDIDATES)]
    table = _time_interleaved(desc, dbuf, cands, reps, rounds, verbose, " global")
    best = _pick(table, margin)
    detail = None
    if per_bucket:
        lanes, unroll, detail = tune_buckets(desc, dbuf, best[0], verbose=verbose)
        combined = best[0][:7] + (tuple(map(tuple, lanes)), tuple(map(tuple, unroll)))
        if combined != best[0]:
            t2 = _time_interleaved(desc, dbuf, [best[0], combined], reps, rounds,
                                   verbose, " combined")
            table = table + [t2[1]]
            if t2[1][1] < t2[0][1] * (1.0 - margin):
                best = t2[1]
    if use_cache:
        cache[sig] = {"tuning": _as_list(best[0]),
                      "table": [[_as_list(c), m] for c, m in table],
                      "buckets": detail, "arch": _arch(), "time": time.time()}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            json.dump(cache, open(tmp, "w"), indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return best[0], table


def tuning_struct(cand):
    return _tuning(cand)


def tune_single_blocks(x, n, dtype, candidates=(0, 256, 384, 512, 768, 1024), reps=20):
    """Time the single-sum kernel at several grid sizes on a device tensor;
    all must agree bit for bit.  Returns (best_blocks, table)."""
    import torch
    from . import new_states, xsum_exact_sum_async_blocks
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = new_states(1)
    sh = stream_handle()
    table, ref = [], None
    for b in candidates:
        for _ in range(3):
            xsum_exact_sum_async_blocks(x.data_ptr(), n, dtype, 255, out.data_ptr(),
                                        fl.data_ptr(), st.data_ptr(), b, sh)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            xsum_exact_sum_async_blocks(x.data_ptr(), n, dtype, 255, out.data_ptr(),
                                        fl.data_ptr(), st.data_ptr(), b, sh)
        e1.record()
        torch.cuda.synchronize()
        r = (int(out.cpu()[0]), int(fl.cpu()[0]))
        if ref is None:
            ref = r
        elif r != ref:
            raise RuntimeError("grid size %d changed the result" % b)
        table.append((b, e0.elapsed_time(e1) / reps))
    return min(table, key=lambda t: t[1])[0], table
