"""Pins of the CPU oracle to things other than itself.

Each test checks the oracle against an independent authority: CPython's
float -> Fraction conversion (exact), CPython's int / int true division
(correctly rounded, OverflowError past the largest double), math.fsum
(correctly rounded sum of doubles), numpy's hardware binary64 -> binary32
conversion (round to nearest even), brute-force Fraction sums, closed forms and
invariants of exact arithmetic.  The planted-mistake tests at the end corrupt
the oracle (on the CPU, in this process only) and check that some pin fails.
"""

import itertools
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import ieee, exact
import workloads

F = oracle.FORMATS
DMAX = np.finfo(np.float64).max
TINY = 5e-324


def d2b(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def b2d(b):
    return struct.unpack("<d", struct.pack("<Q", b))[0]


def cpython_round_f64(total):
    """RNE rounding of total * 2^-1074 to binary64 by CPython's int/int."""
    if total == 0:
        return 0
    try:
        return d2b(total / (1 << 1074))
    except OverflowError:
        return d2b(math.inf if total > 0 else -math.inf)


BOUNDARY_F64 = [0x0, 0x8000000000000000, 0x1, 0x8000000000000001,
                0x000FFFFFFFFFFFFF, 0x0010000000000000, 0x3FF0000000000000,
                0x3FF0000000000001, 0x3FEFFFFFFFFFFFFF, 0x7FEFFFFFFFFFFFFF,
                0xFFEFFFFFFFFFFFFF, 0x0008000000000000, 0x4340000000000000]


# ------------------------------------------------------------------ decode --

def test_decode_f64_matches_fraction():
    rng = np.random.default_rng(1)
    rand = rng.integers(0, 1 << 63, size=3000, dtype=np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, size=3000, dtype=np.uint64)
    pats = BOUNDARY_F64 + [int(b) for b in rand]
    checked = 0
    for b in pats:
        x = b2d(b)
        if not math.isfinite(x):
            assert oracle.decode(b, "f64")[0] in ("inf", "nan")
            continue
        assert exact.value_fraction(b, "f64") == Fraction(x), hex(b)
        checked += 1
    assert checked > 2500


def test_decode_f32_and_bf16_match_fraction():
    rng = np.random.default_rng(2)
    pats32 = [0, 1, 0x80000001, 0x007FFFFF, 0x00800000, 0x3F800000,
              0x7F7FFFFF, 0xFF7FFFFF] + \
        [int(b) for b in rng.integers(0, 1 << 32, size=3000, dtype=np.uint64)]
    for b in pats32:
        x = float(np.array([b], dtype=np.uint32).view(np.float32)[0])
        if not math.isfinite(x):
            continue
        assert exact.value_fraction(b, "f32") == Fraction(x), hex(b)
    for b in range(1 << 16):
        # bfloat16 is the upper half of a binary32
        x = float(np.array([b << 16], dtype=np.uint32).view(np.float32)[0])
        if not math.isfinite(x):
            assert oracle.decode(b, "bf16")[0] in ("inf", "nan")
            continue
        assert exact.value_fraction(b, "bf16") == Fraction(x), hex(b)


# ------------------------------------------------------------------- round --

def _rand_int(rng, nbits):
    """Random Python int with exactly nbits bits (top bit set)."""
    v = 1
    for _ in range(nbits - 1):
        v = (v << 1) | int(rng.integers(0, 2))
    return v


def _round_cases(rng, count):
    vals = []
    for _ in range(count):
        nbits = int(rng.integers(1, 2200))
        v = _rand_int(rng, nbits)
        # also long runs of ones/zeros after the leading bits (near-ties)
        if rng.integers(0, 4) == 0 and nbits > 60:
            cut = int(rng.integers(1, nbits - 1))
            v = (v >> cut << cut) | (((1 << cut) - 1) if rng.integers(0, 2) else 0)
        vals.append(v if rng.integers(0, 2) else -v)
    # exact ties, near-ties, binade edges, subnormal boundary, overflow edges
    for s in (54, 60, 100, 1000, 2000):
        base = (1 << 52 | 12345) << (s - 52)
        half = 1 << (s - 53)
        for off in (0, 1, -1, half, half - 1, half + 1, 2 * half, 3 * half):
            vals += [base + off, -(base + off), base + (1 << (s - 52)) + off]
    top = (1 << 1024 + 1074) - (1 << 970 + 1074)
    vals += [top, top - 1, top + 1, -top, -(top - 1), (1 << 53) - 1, 1 << 53,
             (1 << 53) + 1, (1 << 52) - 1, 1 << 52, 1, 2, 3, (1 << 54) - 1]
    return vals


def test_round_f64_matches_cpython_division():
    rng = np.random.default_rng(3)
    for v in _round_cases(rng, 20000):
        bits, flags = oracle.round_to_format(v, "f64")
        assert bits == cpython_round_f64(v), v
        exact_val = Fraction(v, 1 << 1074)
        if math.isfinite(b2d(bits)):
            assert bool(flags & oracle.FLAG_INEXACT) == (Fraction(b2d(bits)) != exact_val)
            assert not flags & oracle.FLAG_OVERFLOW
        else:
            assert flags & oracle.FLAG_OVERFLOW


def _f32_from_bits(b):
    return float(np.array([b], dtype=np.uint32).view(np.float32)[0])


def _f32_neighbours(x64):
    """binary32 values around the double x64 (numpy nextafter in float32)."""
    with np.errstate(over="ignore"):
        c = np.float32(x64)
    out = {c}
    lo = hi = c
    for _ in range(2):
        lo = np.nextafter(lo, np.float32(-np.inf))
        hi = np.nextafter(hi, np.float32(np.inf))
        out |= {lo, hi}
    return [v for v in out if np.isfinite(v)]


def test_round_f32_matches_hardware_and_neighbour_search():
    rng = np.random.default_rng(4)
    # values with at most 53 significant bits: the double is exact, and the
    # hardware binary64 -> binary32 conversion rounds to nearest even
    for _ in range(20000):
        nb = int(rng.integers(1, 54))
        m = int(rng.integers(1 << (nb - 1), 1 << nb)) if nb > 1 else 1
        sh = int(rng.integers(0, 1300))
        v = m << sh
        if rng.integers(0, 2):
            v = -v
        x = float(Fraction(v, 1 << 1074))       # exact: <= 53 bits
        with np.errstate(over="ignore"):
            want = int(np.array([x], dtype=np.float64).astype(np.float32).view(np.uint32)[0])
        got, flags = oracle.round_to_format(v, "f32")
        assert got == want, (v, hex(got), hex(want))
    # long values: brute force over binary32 neighbours by exact distance
    for _ in range(3000):
        nb = int(rng.integers(54, 200))
        v = _rand_int(rng, nb)
        sh = int(rng.integers(0, 1150))
        v <<= sh
        ex = Fraction(v, 1 << 1074)
        if ex > Fraction(2) ** 128:
            continue
        cands = sorted(set(_f32_neighbours(float(ex))), key=float)
        best = min(cands, key=lambda c: (abs(Fraction(float(c)) - ex),
                                         int(np.array([c], dtype=np.float32).view(np.uint32)[0]) & 1))
        want = int(np.array([best], dtype=np.float32).view(np.uint32)[0])
        got, _ = oracle.round_to_format(v, "f32")
        assert got == want, v


def test_round_bf16_matches_torch_for_f32_exact_values():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    vals = []
    for _ in range(5000):
        nb = int(rng.integers(1, 25))
        m = int(rng.integers(1 << (nb - 1), 1 << nb)) if nb > 1 else 1
        sh = int(rng.integers(930, 1202 - nb))   # binary32 range, 24 bits
        vals.append(-(m << sh) if rng.integers(0, 2) else m << sh)
    xs = np.array([float(Fraction(v, 1 << 1074)) for v in vals], dtype=np.float64)
    f32 = xs.astype(np.float32)
    assert np.all(f32.astype(np.float64) == xs)   # exact in binary32
    want = torch.from_numpy(f32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    for v, w in zip(vals, want.tolist()):
        got, _ = oracle.round_to_format(v, "bf16")
        assert got == w, (v, hex(got), hex(w))


# ---------------------------------------------------------------- whole sum --

@pytest.mark.parametrize("kind", ["positive", "mixed", "anderson", "zero_sum"])
@pytest.mark.parametrize("delta", [10, 200, 2000])
def test_sum_matches_fsum_on_paper_families(kind, delta):
    bits = workloads.family(kind, 4001, delta, seed=delta)
    x = bits.view(np.float64)
    want = d2b(math.fsum(x.tolist())) if math.fsum(x.tolist()) != 0 else 0
    got, _ = oracle.oracle_sum(bits, "f64")
    assert got == want
    got_b, _ = oracle.oracle_sum_binned(bits, "f64", threads=3)
    assert got_b == want


def test_sum_matches_fsum_config1_sample():
    bits = workloads.config1(200_000, seed=11)
    want = d2b(math.fsum(bits.view(np.float64).tolist()))
    assert oracle.oracle_sum(bits, "f64")[0] == want
    assert oracle.oracle_sum_binned(bits, "f64")[0] == want


SPECIAL_SET = [0.0, -0.0, TINY, -TINY, 2 * TINY, 3 * TINY, b2d(0x000FFFFFFFFFFFFF),
               -b2d(0x000FFFFFFFFFFFFF), b2d(0x0010000000000000), 1.0, -1.0,
               1.5, 2.0 ** -53, -(2.0 ** -53), 3 * 2.0 ** -53, 2.0 ** -52,
               1.0 + 2.0 ** -52, -(1.0 + 2.0 ** -52), 2.0 ** 52, 2.0 ** 53, -(2.0 ** 53),
               DMAX, -DMAX, 2.0 ** 970, -(2.0 ** 970), 2.0 ** 1023, -(2.0 ** 1023),
               2.0 ** 971, 0.1, -0.1, 1e-300, -1e-300, 1e300, 3.0, -7.0, 2.0 ** -1022,
               -(2.0 ** -1022), 2.0 ** -1023, 1.0 - 2.0 ** -53, 2.0 ** 1000]


def _fraction_result(vals):
    s = exact.fraction_sum(vals)
    if s == 0:
        return 0
    try:
        return d2b(s.numerator / s.denominator)
    except OverflowError:
        return d2b(math.inf if s > 0 else -math.inf)


def test_bruteforce_fraction_all_pairs_and_random_triples():
    for r in (1, 2):
        for combo in itertools.combinations_with_replacement(SPECIAL_SET, r):
            bits = np.array(combo, dtype=np.float64).view(np.uint64)
            assert oracle.oracle_sum(bits, "f64")[0] == _fraction_result(combo), combo
    rng = np.random.default_rng(6)
    for _ in range(4000):
        combo = [SPECIAL_SET[i] for i in rng.integers(0, len(SPECIAL_SET), size=int(rng.integers(3, 7)))]
        bits = np.array(combo, dtype=np.float64).view(np.uint64)
        assert oracle.oracle_sum(bits, "f64")[0] == _fraction_result(combo), combo


def test_bruteforce_fraction_f32_inputs():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        b = rng.integers(0, 1 << 32, size=int(rng.integers(1, 6)), dtype=np.uint64).astype(np.uint32)
        x = b.view(np.float32)
        if not np.all(np.isfinite(x)):
            continue
        s = exact.fraction_sum([float(v) for v in x])
        want, _ = exact.fraction_to_format(s, "f32")
        # fraction_to_format uses the oracle's rounding; pin it through the
        # neighbour search instead when the sum is not double-exact
        got, _ = oracle.oracle_sum(b, "f32")
        if s == 0:
            assert got == 0
            continue
        if s.denominator & (s.denominator - 1) == 0 and abs(s) < 2 ** 128:
            cands = _f32_neighbours(float(s))
            best = min(cands, key=lambda c: (abs(Fraction(float(c)) - s),
                                             int(np.array([c], dtype=np.float32).view(np.uint32)[0]) & 1))
            assert got == int(np.array([best], dtype=np.float32).view(np.uint32)[0])
        assert got == want


# ----------------------------------------------------- closed forms, invariants --

def test_cancelling_pairs_give_positive_zero():
    a = workloads.config1(5000, seed=12)
    bits = np.concatenate([a, a ^ np.uint64(1 << 63)])
    np.random.default_rng(0).shuffle(bits)
    assert oracle.oracle_sum(bits, "f64") == (0, 0)
    assert oracle.oracle_sum_binned(bits, "f64") == (0, 0)


def test_set_equality_reduction():
    rng = np.random.default_rng(8)
    C = rng.integers(1, 60, size=64)
    D = rng.permutation(C)
    bits, tau = workloads.set_equality(C, D)
    assert oracle.oracle_sum(bits, "f64") == (0, 0)
    # one mismatch leaves exactly 2^(tau d) - 2^(tau c)
    D2 = D.copy()
    D2[5] = 61 if D2[5] != 61 else 62
    bits, tau = workloads.set_equality(C, D2)
    want = d2b(2.0 ** (tau * int(D2[5])) - 2.0 ** (tau * int(D[5])))
    assert oracle.oracle_sum(bits, "f64")[0] == want


def test_k_copies_is_k_times_x():
    rng = np.random.default_rng(9)
    for _ in range(300):
        x = b2d(int(rng.integers(0, 0x7FE0000000000000)))
        k = int(rng.integers(1, 5000))
        bits = np.full(k, d2b(x), dtype=np.uint64)
        assert oracle.oracle_sum(bits, "f64")[0] == _k_times(x, k), (x, k)


def _k_times(x, k):
    s = Fraction(x) * k
    if s == 0:
        return 0
    try:
        return d2b(s.numerator / s.denominator)
    except OverflowError:
        return d2b(math.inf)


def test_permutation_sign_and_scaling_invariance():
    rng = np.random.default_rng(10)
    for trial in range(20):
        bits = workloads.family("mixed", 3000, 400, seed=100 + trial)
        r, _ = oracle.oracle_sum(bits, "f64")
        perm = bits.copy()
        rng.shuffle(perm)
        assert oracle.oracle_sum(perm, "f64")[0] == r
        neg, _ = oracle.oracle_sum(bits ^ np.uint64(1 << 63), "f64")
        assert neg == (r ^ (1 << 63) if r else 0)
        j = int(rng.integers(-300, 300))
        scaled = np.ldexp(bits.view(np.float64), j).view(np.uint64)
        rs, _ = oracle.oracle_sum(scaled, "f64")
        assert b2d(rs) == math.ldexp(b2d(r), j)


def test_config2_closed_form_small():
    bits, terms = workloads.config2(log2n=16, seed=3)
    full = oracle.exact_sum(bits, "f64").total
    assert full == oracle.exact_sum(terms, "f64").total
    assert full != 0
    bits_b, terms_b = workloads.config2(log2n=16, seed=3, variant="b")
    assert oracle.exact_sum(bits_b, "f64").total == oracle.exact_sum(terms_b, "f64").total


def test_special_values_follow_ieee_addition():
    """With small finite parts, the kind of the result (NaN / +inf / -inf)
    matches IEEE addition as numpy performs it."""
    rng = np.random.default_rng(13)
    pool = [np.nan, np.inf, -np.inf, 1.0, -2.5, 0.0, TINY]
    for _ in range(500):
        vals = [pool[i] for i in rng.integers(0, len(pool), size=int(rng.integers(1, 5)))]
        with np.errstate(invalid="ignore"):
            ref = float(np.sum(np.array(vals)))
        got, flags = oracle.oracle_sum(np.array(vals).view(np.uint64), "f64")
        g = b2d(got)
        if math.isnan(ref):
            assert math.isnan(g) and flags & oracle.FLAG_NAN
        elif math.isinf(ref):
            assert g == ref and flags & oracle.FLAG_INF
        else:
            assert g == ref or (g == 0 and ref == 0)


# ---------------------------------------------------------- binned vs loop --

@pytest.mark.parametrize("fmt", ["f64", "f32", "bf16"])
def test_binned_matches_plain_loop(fmt):
    rng = np.random.default_rng(14)
    width = {"f64": 64, "f32": 32, "bf16": 16}[fmt]
    dt = {"f64": np.uint64, "f32": np.uint32, "bf16": np.uint16}[fmt]
    for trial in range(6):
        n = int(rng.integers(0, 200_000))
        bits = rng.integers(0, 1 << width, size=n, dtype=np.uint64).astype(dt)
        if trial % 2 == 0:   # mostly finite
            bits &= dt(~(1 << (width - 2)) & ((1 << width) - 1))
        a = oracle.exact_sum(bits, fmt)
        b, _ = oracle.exact_sum_binned(bits, fmt, threads=1 + trial)
        assert (a.total, a.nan, a.pinf, a.ninf) == (b.total, b.nan, b.pinf, b.ninf)


def _segment_buffer(rng, specs):
    """A byte buffer holding segments of the given (format, bit patterns),
    each at an element-aligned offset after a random gap."""
    chunks, offs, lens, fmts = [], [], [], []
    at = 0
    for fc, bits in specs:
        esize = [8, 4, 2][fc]
        gap = int(rng.integers(0, 5)) * esize
        at += gap
        chunks.append(np.zeros(gap, dtype=np.uint8))
        raw = bits.view(np.uint8)
        offs.append(at)
        lens.append(len(bits))
        fmts.append(fc)
        chunks.append(raw)
        at += raw.size
    return np.concatenate(chunks) if chunks else np.zeros(0, np.uint8), offs, lens, fmts


def test_segmented_sums_match_plain_loop_per_segment():
    # every bit pattern of every format, specials included, at full exponent
    # range: the C fold into wide limbs must give the plain loop's integer
    rng = np.random.default_rng(21)
    width = [64, 32, 16]
    dts = [np.uint64, np.uint32, np.uint16]
    specs = []
    for i in range(60):
        fc = i % 3
        n = int(rng.integers(0, 3000)) if i % 7 else 0
        bits = rng.integers(0, 1 << width[fc], size=n, dtype=np.uint64).astype(dts[fc])
        if i % 2 == 0:   # mostly finite
            bits &= dts[fc](~(1 << (width[fc] - 2)) & ((1 << width[fc]) - 1))
        specs.append((fc, bits))
    # totals near both ends of the range: many +-DBL_MAX, subnormals only
    specs.append((0, np.full(4096, 0x7FEFFFFFFFFFFFFF, dtype=np.uint64)))
    specs.append((0, np.full(4097, 0xFFEFFFFFFFFFFFFF, dtype=np.uint64)))
    specs.append((0, np.arange(1, 5000, dtype=np.uint64)))
    specs.append((1, np.full(3000, 0xFF7FFFFF, dtype=np.uint32)))
    buf, offs, lens, fmts = _segment_buffer(rng, specs)
    got = oracle.segmented_exact_sums(buf, offs, lens, fmts, threads=3)
    names = ["f64", "f32", "bf16"]
    for (fc, bits), g in zip(specs, got):
        a = oracle.exact_sum(bits, names[fc])
        assert (g.total, g.nan, g.pinf, g.ninf) == (a.total, a.nan, a.pinf, a.ninf)
    res = oracle.segmented_oracle_sums(buf, offs, lens, fmts, threads=2)
    for (fc, bits), r in zip(specs, res):
        assert r == tuple(oracle.oracle_sum(bits, names[fc]))


def test_segmented_sums_reject_bad_segments():
    buf = np.zeros(64, dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle.segmented_exact_sums(buf, [0], [9], [0])        # past the end
    with pytest.raises(ValueError):
        oracle.segmented_exact_sums(buf, [0], [1], [3])        # unknown format
    assert oracle.segmented_exact_sums(buf, [], [], []) == []


# -------------------------------------------------------- planted mistakes --

def test_planted_dropped_hidden_bit_is_caught(monkeypatch):
    real = ieee.decode

    def broken(bits, fmt):
        kind, s, m, q = real(bits, fmt)
        if kind == "finite" and m >= (1 << ieee.fmt_of(fmt).t):
            m -= 1 << ieee.fmt_of(fmt).t
        return kind, s, m, q

    monkeypatch.setattr(exact, "decode", broken)
    bits = workloads.config1(2000, seed=15)
    want = d2b(math.fsum(bits.view(np.float64).tolist()))
    assert oracle.oracle_sum(bits, "f64")[0] != want


def test_planted_wrong_sign_is_caught(monkeypatch):
    real = ieee.decode
    monkeypatch.setattr(exact, "decode", lambda b, f: (lambda r: (r[0], 0, r[2], r[3]))(real(b, f)))
    a = workloads.config1(500, seed=16)
    bits = np.concatenate([a, a ^ np.uint64(1 << 63)])
    assert oracle.oracle_sum(bits, "f64") != (0, 0)


def test_planted_ties_away_is_caught(monkeypatch):
    def ties_away(total, fmt):
        f = ieee.fmt_of(fmt)
        a = abs(total)
        top = a.bit_length() - 1
        q = max(top - (f.precision - 1), f.qmin)
        if q > 0 and (a >> (q - 1)) & 1:
            a += 1 << (q - 1)      # round half away from zero
            a -= a & ((1 << q) - 1)
        return ieee.round_to_format(a if total >= 0 else -a, fmt)

    mismatches = 0
    for v in _round_cases(np.random.default_rng(17), 200):
        if ties_away(v, "f64")[0] != cpython_round_f64(v):
            mismatches += 1
    assert mismatches > 0
