"""GPU parity of the single exact sum (xsum_exact_sum, xsum_exact_sum_async)
against the CPU oracle, bit for bit, including the flags."""

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import gpu_sum, gpu_sum_async, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401
    oracle.build_binned(force=False)


def want(bits, fmt, out_fmt=None):
    if len(bits) <= 300_000:
        return tuple(oracle.oracle_sum(bits, fmt, out_fmt))
    return tuple(oracle.oracle_sum_binned(bits, fmt, out_fmt))


@pytest.mark.parametrize("case", workloads.crafted_cases(), ids=lambda c: c[0])
def test_crafted(case):
    name, fmt, bits = case
    print("case", name, flush=True)
    assert gpu_sum(bits, fmt) == want(bits, fmt)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 17, 255, 1023, 4095, 4096, 4097,
                               65537, 100_003, 262_147])
@pytest.mark.parametrize("offset", [0, 1])
def test_ragged_lengths_and_misaligned_start(n, offset):
    bits = workloads.family("mixed", n, 2000, seed=n)
    assert gpu_sum(bits, "f64", offset_elems=offset) == want(bits, "f64")


@pytest.mark.parametrize("kind", ["positive", "mixed", "anderson", "zero_sum"])
@pytest.mark.parametrize("delta", [10, 200, 2000])
def test_paper_families_f64(kind, delta):
    bits = workloads.family(kind, 200_001, delta, seed=7 * delta)
    assert gpu_sum(bits, "f64") == want(bits, "f64")


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["positive", "mixed", "zero_sum"])
@pytest.mark.parametrize("n", [1, 7, 4099, 250_001])
@pytest.mark.parametrize("offset", [0, 3])
def test_narrow_formats(fmt, kind, n, offset):
    bits = workloads.family(kind, n, 250, seed=n + 13, fmt=fmt)
    assert gpu_sum(bits, fmt, offset_elems=offset) == want(bits, fmt)
    # a single rounding straight to binary64 as well
    assert gpu_sum(bits, fmt, out_fmt="f64") == want(bits, fmt, "f64")


@pytest.mark.parametrize("out_fmt", ["f64", "f32", "bf16"])
def test_output_formats_round_once(out_fmt):
    for seed in range(6):
        bits = workloads.family("mixed", 50_000, 120 + 300 * seed, seed=seed)
        assert gpu_sum(bits, "f64", out_fmt) == want(bits, "f64", out_fmt)


def test_random_bit_patterns_with_specials():
    rng = np.random.default_rng(21)
    for fmt, width, dt in (("f64", 64, np.uint64), ("f32", 32, np.uint32),
                           ("bf16", 16, np.uint16)):
        for trial in range(8):
            n = int(rng.integers(1, 70_000))
            bits = rng.integers(0, 1 << width, size=n, dtype=np.uint64).astype(dt)
            if trial < 6:  # mostly finite, so the finite result is exercised
                emax = {64: 0x7FF0000000000000, 32: 0x7F800000, 16: 0x7F80}[width]
                sp = (bits & dt(emax)) == dt(emax)
                bits[sp] ^= dt(1 << (width - 2))
            assert gpu_sum(bits, fmt) == want(bits, fmt), (fmt, trial)


def test_config1_full():
    bits = workloads.config1()
    assert gpu_sum(bits, "f64") == want(bits, "f64")


def test_grid_size_does_not_change_bits():
    bits = workloads.family("mixed", 1_000_003, 2000, seed=99)
    ref = want(bits, "f64")
    t = to_device(bits)
    for blocks in (0, 1, 2, 3, 7, 64, 255, 256, 1000, 5000):
        v, f, state = gpu_sum_async(t, len(bits), "f64", blocks=blocks)
        assert (v, f) == ref, blocks
        assert state == bytes(576), "scratch state must be left zeroed"


def test_async_reuses_scratch_and_sizes_shrink():
    import paper_1605_05436_amd as xs
    st = xs.new_states(1)
    for n in (300_001, 1_000, 17, 0, 5):
        bits = workloads.config1(n, seed=n)
        v, f, state = gpu_sum_async(to_device(bits), n, "f64", scratch=st)
        assert (v, f) == want(bits, "f64")
        assert state == bytes(576)


@pytest.mark.parametrize("fmt,kind", [("f64", "mixed"), ("f64", "zero_sum"),
                                      ("f32", "mixed"), ("bf16", "positive")])
def test_large_inputs_many_blocks(fmt, kind):
    """Every block publishes its partial digits to the scratch state with
    system-scope atomics and the last one rounds: the bits do not depend on
    the grid, and the state is left zero."""
    bits = workloads.family(kind, 2_000_003, 200 if fmt != "f64" else 2000, seed=31, fmt=fmt)
    ref = want(bits, fmt)
    t = to_device(bits)
    for blocks in (0, 3, 977, 4000):
        v, f, state = gpu_sum_async(t, len(bits), fmt, blocks=blocks)
        assert (v, f) == ref, blocks
        assert state == bytes(576), blocks


@pytest.mark.parametrize("pattern", ["positive", "negative", "alternating"])
def test_bfloat16_column_flush(pattern):
    """bfloat16 columns hold 32-bit entries that each wave clears into the
    block vector every 256 tiles.  With one block, 2^23 copies of the value
    whose chunk is the largest possible (significand all ones, shifted by 7)
    put 682 tiles of chunks into the same entry: without the flushes the
    entry would overflow after 2^17 of them."""
    n = 1 << 23
    bits = np.full(n, 0x41ff, dtype=np.uint16)          # 31.875: exponent 131, (131+4) & 7 == 7
    if pattern == "negative":
        bits |= np.uint16(0x8000)
    elif pattern == "alternating":
        bits[1::2] |= np.uint16(0x8000)
        bits[-1] = np.uint16(0x3f80)                    # and a 1.0 so the sum is not zero
    ref = want(bits, "bf16")
    t = to_device(bits)
    for blocks in (1, 0):
        v, f, state = gpu_sum_async(t, n, "bf16", blocks=blocks)
        assert (v, f) == ref, blocks
        assert state == bytes(576)


def test_specials_published_by_distant_blocks():
    """Special values seen by blocks far apart all reach the result; one
    scratch state serves calls of shrinking sizes, the empty sum included."""
    import paper_1605_05436_amd as xs
    st = xs.new_states(1)
    rng = np.random.default_rng(3)
    for n in (1_500_007, 300_001, 4_097, 17, 0):
        bits = workloads.family("mixed", n, 2000, seed=n)
        if n > 100:
            pos = rng.choice(n, size=2, replace=False)
            bits[pos[0]] = np.uint64(0x7ff0000000000000)           # +inf
            if n % 2:
                bits[pos[1]] = np.uint64(0xfff0000000000000)       # -inf -> NaN
        v, f, state = gpu_sum_async(to_device(bits), n, "f64", scratch=st)
        assert (v, f) == want(bits, "f64"), n
        assert state == bytes(576)


def test_carry_stress_many_max_values():
    dmax = workloads.DBL_MAX_BITS
    bits = np.full(1_000_000, dmax, dtype=np.uint64)
    bits[1::2] |= np.uint64(1 << 63)
    bits[-1] = np.uint64(1)                      # + min subnormal
    bits = np.concatenate([bits, np.full(999, dmax, dtype=np.uint64)])
    assert gpu_sum(bits, "f64") == want(bits, "f64")


def test_set_equality_reduction():
    rng = np.random.default_rng(5)
    C = rng.integers(1, 60, size=5000)
    D = rng.permutation(C)
    bits, _ = workloads.set_equality(C, D)
    assert gpu_sum(bits, "f64") == (0, 0)
    D[17] = 63 if D[17] != 63 else 62
    bits, _ = workloads.set_equality(C, D)
    assert gpu_sum(bits, "f64") == want(bits, "f64")


def test_graph_capture_replays_match_eager():
    """The asynchronous sum captured in a graph (its scratch state returns to
    zero after every launch and no memset node is recorded) gives the eager
    result on every replay, with eager library work and synchronisations
    between the replays."""
    import torch
    import paper_1605_05436_amd as xs
    bits = workloads.family("anderson", 3_000_001, 2000, seed=12)
    expect = want(bits, "f64")
    x = to_device(bits)
    other = workloads.family("mixed", 100_003, 200, seed=13)
    xo = to_device(other)
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = xs.new_states(1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        xs.xsum_exact_sum_async(x.data_ptr(), len(bits), xs.F64, xs.F64, out.data_ptr(),
                                fl.data_ptr(), st.data_ptr(), xs.stream_handle(s))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        xs.xsum_exact_sum_async(x.data_ptr(), len(bits), xs.F64, xs.F64, out.data_ptr(),
                                fl.data_ptr(), st.data_ptr(), xs.stream_handle(s))
    for rep in range(4):
        out.fill_(0)
        fl.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (int(out.cpu().numpy().view(np.uint64)[0]), int(fl.cpu()[0]))
        assert got == expect, rep
        assert st.cpu().numpy().tobytes() == bytes(576)
        # eager work on another stream and tensor between the replays
        assert xs.exact_sum(xo, xs.F64) == want(other, "f64")

