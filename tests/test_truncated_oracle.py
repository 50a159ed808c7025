"""Pins of the oracle's Section 4 pass (r-truncated sparse superaccumulators,
the stopping test and r <- r^2) to things other than itself: CPython's exact
float -> Fraction conversion, math.fsum (a correctly rounded sum of doubles),
Fraction brute force, the exact sum oracle (pinned on its own in
test_oracle_pins.py), and the invariants the paper states: regularised
mantissas after every addition, truncation loses less than one unit of the
lowest kept component, the root lies within the summed bound of the exact
sum, and a passing stopping test of the paper gives a faithful rounding."""

import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import truncated as T
import workloads

R = T.R
UNIT = Fraction(1, 1 << 1074)


def d2b(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def b2d(b):
    return struct.unpack("<d", struct.pack("<Q", b))[0]


def exact_units(values):
    """Exact sum of Python floats in units of 2^-1074 through Fraction."""
    s = sum((Fraction(v) for v in values), Fraction(0)) / UNIT
    assert s.denominator == 1
    return s.numerator


def fsum_bits(values):
    s = math.fsum(values)
    return 0 if s == 0 else d2b(s)


def _regularised(y):
    return all(-(R - 1) <= v <= R - 1 for v in y.values())


def _random_sparse(rng, count, lo=0, hi=70, extreme=False):
    y = {}
    for i in rng.choice(np.arange(lo, hi), size=count, replace=False):
        if extreme and rng.random() < 0.5:
            y[int(i)] = int(rng.choice([R - 1, -(R - 1), R - 2, -(R - 2), 1, -1, 0]))
        else:
            y[int(i)] = int(rng.integers(-(R - 1), R))
    return y


# ---------------------------------------------------------------- leaves --

def test_leaf_value_matches_fraction():
    rng = np.random.default_rng(1)
    pats = rng.integers(0, 1 << 63, size=3000, dtype=np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, size=3000, dtype=np.uint64)
    for b in [0, 1, 0x8000000000000001, 0x7FEFFFFFFFFFFFFF, 0x000FFFFFFFFFFFFF] + [int(p) for p in pats]:
        x = b2d(b)
        if not math.isfinite(x):
            assert T.leaf(b, "f64") is None
            continue
        lf = T.leaf(b, "f64")
        assert _regularised(lf) and all(v != 0 for v in lf.values())
        assert T.value(lf) == Fraction(x) / UNIT
        # a binary64 mantissa shifted within one radix digit spans at most 3
        assert len(lf) <= 3


def test_leaf_f32_and_bf16_values():
    rng = np.random.default_rng(2)
    b32 = rng.integers(0, 1 << 32, size=2000, dtype=np.uint64).astype(np.uint32)
    for b, x in zip(b32.tolist(), b32.view(np.float32).tolist()):
        lf = T.leaf(b, "f32")
        if not math.isfinite(x):
            assert lf is None
        else:
            assert T.value(lf) == Fraction(x) / UNIT and len(lf) <= 2
    for h in range(0, 1 << 16, 7):
        x = np.array([h << 16], dtype=np.uint32).view(np.float32)[0]
        lf = T.leaf(h, "bf16")
        if not np.isfinite(x):
            assert lf is None
        else:
            assert T.value(lf) == Fraction(float(x)) / UNIT and len(lf) <= 2


# -------------------------------------------------------------- addition --

def test_carry_add_is_exact_and_regularised():
    rng = np.random.default_rng(3)
    for trial in range(3000):
        y = _random_sparse(rng, int(rng.integers(0, 12)), extreme=trial % 2 == 0)
        z = _random_sparse(rng, int(rng.integers(0, 12)), extreme=trial % 3 == 0)
        s = T.carry_add(y, z)
        assert T.value(s) == T.value(y) + T.value(z)
        assert _regularised(s)
        # active indices stay active; carries add at most the next index up
        assert set(y) | set(z) <= set(s) <= set(y) | set(z) | {i + 1 for i in set(y) | set(z)}


def test_carry_add_extreme_runs_keep_carries_local():
    # every component at the regularisation limit: P_i = 2R - 2 everywhere
    y = {i: R - 1 for i in range(10)}
    s = T.carry_add(y, y)
    assert T.value(s) == 2 * T.value(y) and _regularised(s)
    y = {i: -(R - 1) for i in range(10)}
    s = T.carry_add(y, dict(y))
    assert T.value(s) == 2 * T.value(y) and _regularised(s)


# ------------------------------------------------------------ truncation --

def test_truncation_keeps_top_entries_and_loses_less_than_a_unit():
    rng = np.random.default_rng(4)
    for _ in range(2000):
        y = _random_sparse(rng, int(rng.integers(1, 20)))
        r = int(rng.choice([1, 2, 4, 16]))
        kept, bound = T.truncate(y, r)
        top = sorted(y, reverse=True)[:r]
        assert sorted(kept, reverse=True) == top and all(kept[i] == y[i] for i in top)
        lost = T.value(y) - T.value(kept)
        if bound == 0:
            assert lost == 0
        else:
            assert abs(lost) < bound == R ** min(kept)


@pytest.mark.parametrize("r", [2, 4, 16])
def test_tree_root_within_summed_bound_of_exact_sum(r):
    rng = np.random.default_rng(5 + r)
    for trial in range(60):
        n = int(rng.integers(1, 200))
        kind = ["positive", "mixed", "anderson", "zero_sum"][trial % 4]
        bits = workloads.family(kind, n, int(rng.choice([5, 60, 600])), seed=trial)
        xs = bits.view(np.float64).tolist()
        root, bound = T.tree_sum([T.leaf(b, "f64") for b in bits.tolist()], r)
        assert _regularised(root) and len(root) <= r
        assert abs(exact_units(xs) - T.value(root)) <= bound


# --------------------------------------------------------- stopping test --

def test_certified_results_are_the_rne_rounding():
    rng = np.random.default_rng(6)
    for _ in range(3000):
        total = int(rng.integers(-(1 << 62), 1 << 62)) << int(rng.integers(0, 1100))
        bound = int(rng.integers(0, 1 << 40)) << int(rng.integers(0, 1100))
        res = T.certified(total, bound, "f64")
        if res is None:
            continue
        for probe in (total - bound, total, total + bound):
            assert oracle.round_to_format(probe, "f64")[0] == res[0]
        if bound:
            assert res[1] & oracle.FLAG_INEXACT


def test_certified_refuses_an_interval_around_a_tie_or_a_float():
    one = 1 << 1074                      # 1.0 in units of 2^-1074
    half_ulp = 1 << (1074 - 53)
    # 1 + 2^-53 is a tie between 1 and 1 + 2^-52; any bound straddles it
    assert T.certified(one + half_ulp, 1, "f64") is None
    # the interval contains the float 1.0 itself: exactness is undecided
    assert T.certified(one, 1, "f64") is None
    assert T.certified(one + 1, 2, "f64") is None
    # clear of both: rounds to 1.0, inexact
    assert T.certified(one + 10, 2, "f64") == (d2b(1.0), oracle.FLAG_INEXACT)
    # no truncation: the exact rounding, exact flag
    assert T.certified(one, 0, "f64") == (d2b(1.0), 0)
    # an interval across zero never certifies
    assert T.certified(0, 1, "f64") is None


def _faithful(bits, values):
    """bits is one of the two doubles around the exact sum of values."""
    y = b2d(bits)
    if not math.isfinite(y):
        return True
    e = sum((Fraction(v) for v in values), Fraction(0))
    lo, hi = math.nextafter(y, -math.inf), math.nextafter(y, math.inf)
    return Fraction(lo) < e < Fraction(hi) if math.isfinite(lo) and math.isfinite(hi) else True


def test_paper_stopping_tests_give_faithful_roundings():
    rng = np.random.default_rng(7)
    passed = [0, 0]
    for trial in range(300):
        n = int(rng.integers(2, 120))
        kind = ["positive", "mixed", "anderson", "zero_sum"][trial % 4]
        bits = workloads.family(kind, n, int(rng.choice([5, 60, 600, 1500])), seed=100 + trial)
        xs = bits.view(np.float64).tolist()
        for r in (2, 4, 16):
            root, _ = T.tree_sum([T.leaf(b, "f64") for b in bits.tolist()], r)
            tests = T.paper_tests(root, n, "f64")
            if any(tests):
                y, _ = oracle.round_to_format(T.value(root), "f64")
                assert _faithful(y, xs), (kind, n, r, tests)
            for i in range(2):
                passed[i] += tests[i]
    assert passed[0] > 50 and passed[1] > 50


# -------------------------------------------------------- whole iteration --

@pytest.mark.parametrize("kind", ["positive", "mixed", "anderson", "zero_sum"])
@pytest.mark.parametrize("delta", [10, 200, 2000])
def test_adaptive_sum_matches_fsum_on_paper_families(kind, delta):
    bits = workloads.family(kind, 1500, delta, seed=delta)
    (got, flags), passes, r = T.adaptive_sum(bits, "f64")
    assert got == fsum_bits(bits.view(np.float64).tolist())
    assert 1 <= passes <= 4 and r == 2 ** (2 ** (passes - 1))


def test_adaptive_sum_matches_exact_oracle_on_workloads():
    for seed in range(3):
        bits = workloads.config1(4000, seed=seed)
        assert T.adaptive_sum(bits, "f64")[0] == tuple(oracle.oracle_sum(bits, "f64"))
    b2, _ = workloads.config2(log2n=11, seed=1)
    assert T.adaptive_sum(b2, "f64")[0] == tuple(oracle.oracle_sum(b2, "f64"))
    for fmt in ("f32", "bf16"):
        rng = np.random.default_rng(8)
        b = rng.integers(0, 1 << 32, size=3000, dtype=np.uint64).astype(np.uint32)
        if fmt == "bf16":
            b = (b >> 16).astype(np.uint16)
        x = b.view(np.float32 if fmt == "f32" else np.uint16)
        if fmt == "f32":
            b = b[np.isfinite(x)]
        else:
            b = b[(b & 0x7F80) != 0x7F80]
        for out in ("f64", "f32", "bf16"):
            assert T.adaptive_sum(b, fmt, out)[0] == tuple(oracle.oracle_sum(b, fmt, out))


def test_adaptive_sum_edge_cases():
    empty = np.zeros(0, dtype=np.uint64)
    assert T.adaptive_sum(empty, "f64")[:2] == ((0, 0), 1)
    zeros = np.array([0.0, -0.0, 0.0]).view(np.uint64)
    assert T.adaptive_sum(zeros, "f64")[0] == (0, 0)
    one = np.array([-2.5]).view(np.uint64)
    assert T.adaptive_sum(one, "f64")[0] == (d2b(-2.5), 0)
    ovf = np.array([np.finfo(np.float64).max] * 2).view(np.uint64)
    assert T.adaptive_sum(ovf, "f64")[0] == tuple(oracle.oracle_sum(ovf, "f64"))
    spec = np.array([1.0, math.inf, -math.inf]).view(np.uint64)
    assert T.adaptive_sum(spec, "f64")[0] == tuple(oracle.oracle_sum(spec, "f64"))
    spec = np.array([1.0, -math.inf]).view(np.uint64)
    assert T.adaptive_sum(spec, "f64")[0] == tuple(oracle.oracle_sum(spec, "f64"))


def test_passes_follow_the_condition_number():
    # equal integers never need truncation beyond two components
    same = np.array([3.0] * 1000).view(np.uint64)
    assert T.adaptive_sum(same, "f64")[1] == 1
    # a well-conditioned sum stops early; heavy cancellation across the
    # exponent range needs the untruncated pass (Theorem 4: O(log log C) passes)
    well = workloads.family("positive", 2000, 10, seed=1)
    # twenty terms 31 bits apart, 1.0, then their negatives: C(X) ~ 2^1000, and
    # the cancelled indices stay active, so only the untruncated pass is exact
    big = [2.0 ** (1000 - 31 * k) for k in range(20)]
    ill = np.array(big + [1.0] + [-v for v in big]).view(np.uint64)
    p_well = T.adaptive_sum(well, "f64")[1]
    (got, flags), p_ill, r = T.adaptive_sum(ill, "f64")
    assert p_well <= 2 and p_ill == 4 and r == 256
    assert (got, flags) == (d2b(1.0), 0)


def test_planted_dropped_carry_is_caught(monkeypatch):
    # a carry_add that forgets the incoming carry breaks the bound pin
    def bad(y, z):
        p = {i: y.get(i, 0) + z.get(i, 0) for i in set(y) | set(z)}
        return {i: pi - (1 if pi >= R - 1 else (-1 if pi <= -(R - 1) else 0)) * R
                for i, pi in p.items()}
    monkeypatch.setattr(T, "carry_add", bad)
    bits = workloads.family("positive", 3000, 3, seed=2)
    (got, _), _, _ = T.adaptive_sum(bits, "f64")
    assert got != fsum_bits(bits.view(np.float64).tolist())
