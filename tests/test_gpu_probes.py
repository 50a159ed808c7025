"""The measurement kernels the benchmark reads its reference points from
(read ceiling, cache eviction, shader clock) do what their declarations say.
They carry none of the summation method."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401


def test_flush_fills_every_word():
    import torch
    import paper_1605_05436_amd as xs
    buf = torch.zeros((1 << 20) + 3, dtype=torch.int32, device="cuda")
    xs.xsum_probe_flush(buf.data_ptr(), buf.numel() * 4, 0x5A5A1234, xs.stream_handle())
    torch.cuda.synchronize()
    assert bool((buf == 0x5A5A1234).all())


def test_read_probe_runs_over_a_ragged_buffer():
    import torch
    import paper_1605_05436_amd as xs
    x = torch.arange(1 << 18, dtype=torch.int64, device="cuda")
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    for nbytes in (16, 48 * 1024 + 16, x.numel() * 8):
        xs.xsum_probe_read(x.data_ptr(), nbytes, sink.data_ptr(), xs.stream_handle())
    torch.cuda.synchronize()


def test_clock_samples_advance_at_the_requested_interval():
    import torch
    import paper_1605_05436_amd as xs
    n, interval = 200, 1000                      # one sample every 10 us
    out = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    xs.xsum_probe_clock(out.data_ptr(), n, interval, xs.stream_handle())
    torch.cuda.synchronize()
    s = out.cpu().numpy().reshape(-1, 2)
    rt, ck = np.diff(s[:, 0]), np.diff(s[:, 1])
    # the constant-rate counter advances by about the interval (a sample can
    # be taken a little late), the shader-clock counter never goes back
    assert (rt > interval // 2).all() and np.median(rt) < 2 * interval
    assert (ck > 0).all()
    mhz = ck / rt * 100.0
    # a plausible shader clock: below the 2.4 GHz peak with margin, and
    # well above the 100 MHz reference while a wave is running
    assert 200 < np.median(mhz) < 3000, mhz
