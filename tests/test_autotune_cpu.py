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
