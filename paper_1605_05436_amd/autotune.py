"""Autotuner for segmented sums and the single-sum grid.

For a batch of segments the tunables decide which path each length bucket
takes and how work is cut: lane_max (per-lane groups below it), wave_max (one
wave per segment below it), chunk_vectors (chunk size above it),
blocks_per_cu (resident one-wave groups per CU) and lane_buckets (length
buckets per doubling inside the per-lane path).  The tuner times candidate
plans on the device with captured-graph replays, checks that every candidate
returns bit-identical results (exactness makes that a hard requirement, not a
tolerance), and keeps the fastest.  Results are cached in a JSON file keyed
by the device architecture and a coarse signature of the batch (per-format
log2-length histogram), so later plans of similar batches reuse them.

The cache path is $XSUM_TUNE_CACHE, else ~/.cache/xsum/tune.json.
"""

import hashlib
import json
import os
import time

import numpy as np

from . import (SegTuning, SegmentedSum, xsum_graph_launch, xsum_graph_destroy,
               stream_handle)

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


def _tuning(c):
    lane, wave, chunk, bpc, buckets = c[:5]
    two, four = c[5:7] if len(c) >= 7 else (0, 0)
    t = SegTuning()
    for d in range(3):
        t.lane_max[d] = lane[d]
        t.wave_max[d] = wave[d]
    t.chunk_vectors = chunk
    t.blocks_per_cu = bpc
    t.lane_buckets = buckets
    t.two_lanes_from = two
    t.four_lanes_from = four
    return t


def _as_list(c):
    return [list(c[0]), list(c[1])] + list(c[2:])


def _from_list(c):
    return (tuple(c[0]), tuple(c[1])) + tuple(c[2:])


def _time_candidate(desc, dbuf, cand, reps, out, flags):
    import torch
    ss = SegmentedSum(desc, tuning=_tuning(cand))
    g = ss.capture(dbuf, out, flags)
    sh = stream_handle()
    try:
        for _ in range(2):
            xsum_graph_launch(g, sh)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            xsum_graph_launch(g, sh)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res = (out.cpu().numpy().copy(), flags.cpu().numpy().copy())
    finally:
        xsum_graph_destroy(g)
        ss.close()
    return ms, res


def tune_segmented(desc, dbuf, candidates=None, reps=5, use_cache=True,
                   verbose=False, margin=0.03):
    """Pick the fastest tuning for this batch.  Returns (tuning tuple, table)
    where table lists (candidate, ms).  Raises if candidates disagree.  The
    first candidate (the library defaults) is kept unless another is faster
    by more than `margin` (relative), so near-ties between timings resolve
    the same way from run to run."""
    import torch
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
    cands = candidates or DEFAULT_CANDIDATES
    out = torch.zeros(len(desc), dtype=torch.int64, device="cuda")
    flags = torch.zeros(len(desc), dtype=torch.int32, device="cuda")
    table, ref, best = [], None, None
    for cand in cands:
        ms, res = _time_candidate(desc, dbuf, cand, reps, out, flags)
        if ref is None:
            ref = res
        elif not (np.array_equal(res[0], ref[0]) and np.array_equal(res[1], ref[1])):
            raise RuntimeError("autotune candidate %r changed the results" % (cand,))
        table.append((cand, ms))
        if verbose:
            print("[autotune] %r: %.3f ms" % (cand, ms), flush=True)
        if best is None or ms < best[1] * (1.0 - margin):
            best = (cand, ms)
    if use_cache:
        cache[sig] = {"tuning": _as_list(best[0]),
                      "table": [[_as_list(c), m] for c, m in table],
                      "arch": _arch(), "time": time.time()}
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
