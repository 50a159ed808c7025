"""The allocation-free segmented run (xsum_segmented_run_noalloc, whose
workspace is the library's per-device static array) gives the same bits as
xsum_segmented_run with a caller workspace, on two calls in a row, the second
with a smaller batch; plans that need more than the array are rejected."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401


def _both(dbuf, desc, tuning=None):
    import torch
    import paper_1605_05436_amd as xs
    ss = xs.SegmentedSum(desc, xs.SAME, tuning)
    n = max(1, len(desc))
    out_a = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    fl_a = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    out_b = torch.full((n,), -2, dtype=torch.int64, device="cuda")
    fl_b = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    ss.run(dbuf, out_a, fl_a)
    xs.xsum_segmented_run_noalloc(ss.plan, dbuf.data_ptr(), out_b.data_ptr(),
                                  fl_b.data_ptr(), xs.stream_handle())
    torch.cuda.synchronize()
    info = ss.info
    ss.close()
    return (out_a.cpu().numpy(), fl_a.cpu().numpy(), out_b.cpu().numpy(),
            fl_b.cpu().numpy(), info)


def test_noalloc_run_matches_workspace_run_twice():
    import torch
    import paper_1605_05436_amd as xs
    lengths = np.concatenate([workloads.segment_lengths(4000, seed=51),
                              [400_000, 1_300_000, 262_145, 1, 0]]).astype(np.int64)
    dtypes = np.concatenate([workloads.segment_dtypes(4000, seed=52),
                             [0, 0, 0, 1, 2]]).astype(np.int64)
    buf, desc = workloads.config4(nseg=len(lengths), seed=53, lengths=lengths,
                                  dtypes=dtypes)
    dbuf = torch.from_numpy(buf).to("cuda")
    # small chunks so that many chunked segments share the static array
    tuning = xs.SegTuning()
    tuning.chunk_vectors = 4096
    for d in range(3):
        tuning.wave_max[d] = 20_000
    a, fa, b, fb, info = _both(dbuf, desc, tuning)
    assert info["chunked_segments"] >= 40
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    # second call, smaller batch, default tuning, same static array
    sub = desc[::5].copy()
    a, fa, b, fb, info = _both(dbuf, sub)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    assert info["chunked_segments"] >= 1


def test_noalloc_run_rejects_plans_beyond_the_array():
    import torch
    import paper_1605_05436_amd as xs
    # 2000 chunked segments need 256 + 2000 * 576 bytes > 1 MiB
    lengths = np.full(2000, 300, dtype=np.int64)
    buf, desc = workloads.config4(nseg=2000, seed=54, lengths=lengths,
                                  dtypes=np.zeros(2000, dtype=np.int64))
    tuning = xs.SegTuning()
    for d in range(3):
        tuning.lane_max[d] = 16
        tuning.wave_max[d] = 64
    tuning.chunk_vectors = 64
    ss = xs.SegmentedSum(desc, xs.SAME, tuning)
    assert ss.info["chunked_segments"] == 2000
    dbuf = torch.from_numpy(buf).to("cuda")
    out = torch.zeros(2000, dtype=torch.int64, device="cuda")
    with pytest.raises(xs.XsumError) as e:
        xs.xsum_segmented_run_noalloc(ss.plan, dbuf.data_ptr(), out.data_ptr(), 0,
                                      xs.stream_handle())
    assert e.value.status == xs.ERANGE
    ss.close()
