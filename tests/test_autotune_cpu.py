"""Host-side parts of the autotuner: the batch signature is stable, depends
on the length distribution, and the cache round-trips."""

import numpy as np

import workloads


def test_signature_is_stable_and_distribution_sensitive():
    from paper_1605_05436_amd import autotune
    L = workloads.segment_lengths(20000, 0)
    D = workloads.segment_dtypes(20000, 0)
    desc = np.zeros(len(L), dtype=workloads.SEGMENT_DTYPE)
    desc["length"], desc["dtype"] = L, D
    s1 = autotune.batch_signature(desc)
    assert s1 == autotune.batch_signature(desc.copy())
    desc2 = desc.copy()
    desc2["length"] = np.maximum(1, desc2["length"] // 64)
    assert autotune.batch_signature(desc2) != s1


def test_tuning_struct_fields():
    from paper_1605_05436_amd import autotune
    t = autotune.tuning_struct(((1, 2, 3), (4, 5, 6), 7, 8, 9))
    assert list(t.lane_max) == [1, 2, 3] and list(t.wave_max) == [4, 5, 6]
    assert (t.chunk_vectors, t.blocks_per_cu, t.lane_buckets) == (7, 8, 9)


def test_tuning_tables_round_trip_through_the_cache_format():
    from paper_1605_05436_amd import autotune
    lanes = [[0] * autotune.NB for _ in range(3)]
    unroll = [[0] * autotune.NB for _ in range(3)]
    lanes[0][11], unroll[0][11] = 8, 16
    lanes[2][5], unroll[2][5] = 1, 8
    c = ((1, 2, 3), (4, 5, 6), 7, 8, 9, 10, 11,
         tuple(map(tuple, lanes)), tuple(map(tuple, unroll)))
    assert autotune._from_list(autotune._as_list(c)) == c
    t = autotune.tuning_struct(c)
    assert t.lanes[0][11] == 8 and t.lane_unroll[2][5] == 8 and t.lanes[1][3] == 0
    assert (t.two_lanes_from, t.four_lanes_from) == (10, 11)
    # short (old) candidates get empty tables
    assert autotune._full(((0, 0, 0), (0, 0, 0), 0, 0, 0))[7] == autotune.EMPTY_TABLE


def test_lane_buckets_follow_the_planner_rule():
    # bucket = floor(log2(length * element size)), lane-group segments only
    from paper_1605_05436_amd import autotune
    desc = np.zeros(6, dtype=workloads.SEGMENT_DTYPE)
    desc["length"] = [1, 3, 256, 257, 20000, 0]
    desc["dtype"] = [0, 1, 0, 2, 0, 1]
    g = autotune.lane_buckets_of(desc, (16384, 16384, 32768))
    assert sorted(g) == [(0, 3), (0, 11), (1, 0), (1, 3), (2, 9)]
    assert list(g[(0, 11)]) == [2] and list(g[(1, 0)]) == [5]
