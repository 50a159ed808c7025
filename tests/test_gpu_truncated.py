"""GPU parity of the Section 4 pass (r-truncated sparse superaccumulators,
the stopping test, r <- r^2) through the C-ABI.

The pass's result is the round-to-nearest-even sum, which is unique: it is
compared bit for bit (with its flags) against the oracle's exact rounding.
Each single pass is checked against what holds for any correct pass: its root
lists at most r entries in decreasing index order, the exact sum (the
oracle's integer) lies within the pass's bound of the root's value, and a
certified pass carries the exact rounding.  Which pass certifies depends on
the tree's shape, which differs from the oracle's balanced tree, so it is
only checked where it is forced: no truncation at all (r = 2 certifies), or
more active indices above the only non-cancelling term than r = 16 keeps
(only the untruncated pass is exact).  The r = 2 and 4 passes keep their
lists in registers and the r = 16 pass in LDS columns, so every test runs
all three passes."""

import numpy as np
import pytest

import oracle
from oracle import truncated as T
import workloads
from tests.gpu_helpers import FMT_CODE, to_device

pytestmark = pytest.mark.gpu

NAMES = ["f64", "f32", "bf16"]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_05436_amd  # noqa: F401


@pytest.fixture(scope="module")
def ws():
    import torch
    import paper_1605_05436_amd as xs
    n = xs.xsum_truncated_workspace_size()
    return torch.zeros(n, dtype=torch.uint8, device="cuda"), n


def run_blocking(t, n, fmt, ws, out_fmt=None):
    import paper_1605_05436_amd as xs
    buf, nbytes = ws
    oc = xs.SAME if out_fmt is None else FMT_CODE[out_fmt]
    return xs.xsum_exact_sum_truncated(t.data_ptr() if n else 0, n, FMT_CODE[fmt], oc,
                                       buf.data_ptr(), nbytes, xs.stream_handle())


def run_pass(t, n, fmt, r, ws, out_fmt=None):
    import torch
    import paper_1605_05436_amd as xs
    buf, nbytes = ws
    rec = torch.zeros(256, dtype=torch.uint8, device="cuda")
    oc = xs.SAME if out_fmt is None else FMT_CODE[out_fmt]
    xs.xsum_truncated_round(t.data_ptr() if n else 0, n, FMT_CODE[fmt], oc, r,
                            rec.data_ptr(), buf.data_ptr(), nbytes, xs.stream_handle())
    torch.cuda.synchronize()
    return xs.read_trunc_root(rec)


def check_pass(rec, r, exact_total, want):
    """What every correct pass satisfies, whatever its tree."""
    assert rec.r == r and rec.count <= r
    idx = [rec.index[j] for j in range(rec.count)]
    assert idx == sorted(idx, reverse=True) and len(set(idx)) == len(idx)
    assert all(rec.index[j] < 0 and rec.value[j] == 0 for j in range(rec.count, 16))
    s = sum(rec.value[j] << (32 * rec.index[j]) for j in range(rec.count))
    bound = rec.bound_value << (32 * rec.bound_index) if rec.bound_value else 0
    if not rec.special:
        assert abs(exact_total - s) <= bound, (r, exact_total - s, bound)
    if rec.certified:
        assert (rec.bits, rec.flags) == want
    if rec.bound_value == 0 and not rec.special:
        # nothing truncated: the root is exact and the pass must certify
        assert rec.certified


def _inputs():
    rng = np.random.default_rng(0)
    cases = []
    for n in (1, 2, 3, 7, 64, 1000, 4099, 70_001):
        cases.append(("config1-%d" % n, "f64", workloads.config1(n, seed=n)))
    b2, _ = workloads.config2(log2n=14, seed=3)
    cases.append(("config2-2^14", "f64", b2))
    for kind in ("positive", "mixed", "anderson", "zero_sum"):
        for delta in (10, 600, 2000):
            cases.append(("%s-%d" % (kind, delta), "f64",
                          workloads.family(kind, 20_011, delta, seed=delta)))
    for kind in ("mixed", "positive", "zero_sum"):
        cases.append(("f32-%s" % kind, "f32", workloads.family(kind, 30_007, 60, seed=1, fmt="f32")))
        cases.append(("bf16-%s" % kind, "bf16", workloads.family(kind, 30_011, 60, seed=2, fmt="bf16")))
    raw = rng.integers(0, 1 << 32, size=50_001, dtype=np.uint64).astype(np.uint32)
    cases.append(("f32-random-bits", "f32", raw[(raw & 0x7F800000) != 0x7F800000]))
    cases.append(("bf16-random-bits", "bf16",
                  (raw >> 16).astype(np.uint16)[((raw >> 16) & 0x7F80) != 0x7F80]))
    return cases


CASES = _inputs()


@pytest.mark.parametrize("name,fmt,bits", CASES, ids=[c[0] for c in CASES])
def test_iteration_matches_oracle(name, fmt, bits, ws):
    print("truncated iteration", name, len(bits), flush=True)
    want = tuple(oracle.oracle_sum(bits, fmt))
    t = to_device(bits)
    got_bits, got_flags, r = run_blocking(t, len(bits), fmt, ws)
    assert (got_bits, got_flags) == want
    assert r in (2, 4, 16, 0)


@pytest.mark.parametrize("name,fmt,bits", CASES[::3], ids=[c[0] for c in CASES[::3]])
def test_every_pass_is_sound(name, fmt, bits, ws):
    print("truncated passes", name, len(bits), flush=True)
    exact = oracle.exact_sum(bits, fmt)
    t = to_device(bits)
    for out_fmt in ("f64", "f32", "bf16"):
        want = tuple(oracle.oracle_sum(bits, fmt, out_fmt))
        for r in (2, 4, 16):
            check_pass(run_pass(t, len(bits), fmt, r, ws, out_fmt), r, exact.total, want)


@pytest.mark.parametrize("offset", [1, 3])
@pytest.mark.parametrize("fmt", NAMES)
def test_unaligned_start_and_ragged_tail(fmt, offset, ws):
    n = 10_007
    bits = workloads.family("mixed", n, 300, seed=offset, fmt=fmt) if fmt != "f64" \
        else workloads.config1(n, seed=offset)
    want = tuple(oracle.oracle_sum(bits, fmt))
    t = to_device(bits, offset_elems=offset)
    assert run_blocking(t, n, fmt, ws)[:2] == want
    exact = oracle.exact_sum(bits, fmt).total
    for r in (2, 16):
        check_pass(run_pass(t, n, fmt, r, ws), r, exact, want)


def test_empty_zero_and_specials(ws):
    import math
    import torch
    e = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert run_blocking(e, 0, "f64", ws) == (0, 0, 2)
    for vals in ([0.0, -0.0, 0.0], [-2.5], [1.0, math.inf], [1.0, math.inf, -math.inf],
                 [math.nan, 1.0], [-math.inf] * 3, [np.finfo(np.float64).max] * 2,
                 [np.finfo(np.float64).max, -np.finfo(np.float64).max, 5e-324]):
        bits = np.array(vals, dtype=np.float64).view(np.uint64)
        want = tuple(oracle.oracle_sum(bits, "f64"))
        t = to_device(bits)
        got = run_blocking(t, len(bits), "f64", ws)
        assert got[:2] == want, vals
        for r in (2, 4, 16):
            rec = run_pass(t, len(bits), "f64", r, ws)
            if any(not math.isfinite(v) for v in vals):
                assert rec.certified and (rec.bits, rec.flags) == want
            else:
                check_pass(rec, r, oracle.exact_sum(bits, "f64").total, want)


def test_pass_count_where_it_is_forced(ws):
    # equal small integers: at most two active indices anywhere, no truncation
    same = np.array([3.0] * 100_000).view(np.uint64)
    t = to_device(same)
    assert run_blocking(t, len(same), "f64", ws) == (tuple(oracle.oracle_sum(same, "f64")) + (2,))
    rec = run_pass(t, len(same), "f64", 2, ws)
    assert rec.bound_value == 0 and rec.certified
    # 20 cancelling terms at distinct indices above 1.0: every tree keeps at
    # most 16 of the active indices, all above 1.0's, so r = 16 cannot hold it
    big = [2.0 ** (1000 - 31 * k) for k in range(20)]
    active = {i for v in big for i in T.leaf(int(np.array([v]).view(np.uint64)[0]), "f64")}
    assert len(active) > 16
    ill = np.array(big + [1.0] + [-v for v in big]).view(np.uint64)
    t = to_device(ill)
    assert run_blocking(t, len(ill), "f64", ws) == (int(np.array([1.0]).view(np.uint64)[0]), 0, 0)
    rec = run_pass(t, len(ill), "f64", 16, ws)
    assert not rec.certified and rec.bound_value > 0


def test_pass_records_do_not_depend_on_scheduling(ws):
    bits = workloads.config1(300_007, seed=5)
    t = to_device(bits)
    for r in (2, 4, 16):
        a = bytes(run_pass(t, len(bits), "f64", r, ws))
        for _ in range(3):
            assert bytes(run_pass(t, len(bits), "f64", r, ws)) == a


@pytest.mark.parametrize("fmt", NAMES)
def test_special_values_inside_tiles(fmt, ws):
    """Infinities and NaNs met in the middle of a lane's tiles (not only in
    the head or tail): every pass records them and certifies the special
    result."""
    n = 200_003
    bits = workloads.family("mixed", n, 60, seed=9, fmt=fmt) if fmt != "f64" \
        else workloads.config1(n, seed=9)
    rng = np.random.default_rng(3)
    allones = {"f64": (0x7FF0000000000000, 0xFFF0000000000000, 0x7FF8000000000001),
               "f32": (0x7F800000, 0xFF800000, 0x7FC00001),
               "bf16": (0x7F80, 0xFF80, 0x7FC1)}[fmt]
    for case in ((0,), (1,), (0, 1), (2,), (0, 0)):
        b = bits.copy()
        at = rng.choice(np.arange(64, n - 64), size=len(case), replace=False)
        for pos, which in zip(at, case):
            b[pos] = allones[which]
        want = tuple(oracle.oracle_sum(b, fmt))
        t = to_device(b)
        assert run_blocking(t, n, fmt, ws)[:2] == want, case
        for r in (2, 4, 16):
            rec = run_pass(t, n, fmt, r, ws)
            assert rec.special and rec.certified and (rec.bits, rec.flags) == want, (case, r)
