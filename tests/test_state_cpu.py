"""The compact state encoding (xsum_state_encode / xsum_state_decode) on the
host: an independent Python reading of the documented byte layout recovers
the exact value of the encoded state; decoding gives canonical digits of the
same value; the digit run is minimal; malformed input is rejected.  No GPU."""

import random
import struct

import numpy as np
import pytest

import oracle
import workloads

DIGITS = 68
MASK = (1 << 32) - 1


@pytest.fixture(scope="module")
def xs():
    try:
        import paper_1605_05436_amd as m
    except ImportError as e:
        pytest.fail("library not built: %s" % e)
    return m


def state_bytes(digits, special=0):
    assert len(digits) == DIGITS
    return (np.array(digits, dtype=np.int64).tobytes() +
            struct.pack("<II", special, 0) + bytes(24))


def state_value(raw):
    d = np.frombuffer(raw[:8 * DIGITS], dtype=np.int64)
    return sum(int(v) << (32 * j) for j, v in enumerate(d.tolist()))


def canonical_digits(value):
    """Digits 0..66 in [0, 2^32) and the signed top digit of an integer."""
    return [(value >> (32 * j)) & MASK for j in range(DIGITS - 1)] + [value >> (32 * (DIGITS - 1))]


def read_encoding(data):
    """Independent reader of the layout in include/xsum.h: returns
    (special, value)."""
    magic, special, sign, lo, cnt, zero = struct.unpack_from("<IIBBBB", data, 0)
    assert magic == 0x31535358 and zero == 0 and sign in (0, 1)
    assert len(data) == 12 + 4 * cnt
    digits = struct.unpack_from("<%dI" % cnt, data, 12)
    if cnt:
        assert digits[0] != 0 and digits[-1] != 0       # minimal run
    mag = sum(d << (32 * (lo + k)) for k, d in enumerate(digits))
    assert not (sign and mag == 0)
    return special, -mag if sign else mag


def random_state(rng):
    kind = rng.random()
    if kind < 0.3:      # arbitrary (non-canonical) digits
        d = [rng.randrange(-(1 << 62), (1 << 62) + 1) for _ in range(DIGITS - 1)]
        d.append(rng.randrange(-(1 << 59), (1 << 59) + 1))
        return d
    if kind < 0.6:      # canonical digits of a random value with a few digits
        lo = rng.randrange(0, 66)
        width = rng.randrange(1, min(6, 67 - lo) + 1)
        v = rng.randrange(1, 1 << (32 * width)) << (32 * lo)
        return canonical_digits(v if rng.random() < 0.5 else -v)
    # sparse raw digits with carries that ripple across many digits
    d = [0] * DIGITS
    for _ in range(rng.randrange(1, 5)):
        d[rng.randrange(0, DIGITS - 1)] += rng.choice([-1, 1]) * rng.randrange(1, 1 << 62)
    d = [max(-(1 << 62), min(1 << 62, x)) for x in d]
    return d


def test_roundtrip_preserves_value_and_is_canonical(xs):
    rng = random.Random(7)
    for i in range(3000):
        digits = random_state(rng)
        special = rng.choice([0, 0, 0, 1, 2, 4, 6, 7])
        raw = state_bytes(digits, special)
        value = state_value(raw)
        enc = xs.xsum_state_encode(raw)
        assert len(enc) <= xs.STATE_ENCODED_MAX
        assert read_encoding(enc) == (special, value), i
        dec = xs.xsum_state_decode(enc)
        assert len(dec) == 576
        assert state_value(dec) == value
        d = np.frombuffer(dec[:8 * DIGITS], dtype=np.int64).tolist()
        assert d == canonical_digits(value)
        assert struct.unpack_from("<II", dec, 8 * DIGITS) == (special, 0)
        assert dec[8 * DIGITS + 8:] == bytes(24)
        assert xs.xsum_state_encode(dec) == enc      # canonical form re-encodes alike


def test_zero_and_extremes(xs):
    z = xs.xsum_state_encode(bytes(576))
    assert len(z) == 12 and read_encoding(z) == (0, 0)
    assert xs.xsum_state_decode(z) == bytes(576)
    # the largest and smallest encodable values
    for v in ((1 << (32 * 67 + 61)) + 12345, -(1 << (32 * 67 + 61)), 1, -1, 1 << 2143):
        raw = state_bytes(canonical_digits(v))
        enc = xs.xsum_state_encode(raw)
        assert read_encoding(enc)[1] == v
        assert state_value(xs.xsum_state_decode(enc)) == v
    with pytest.raises(xs.XsumError) as e:
        xs.xsum_state_encode(state_bytes(canonical_digits(1 << (32 * 67 + 62))))
    assert e.value.status == xs.ERANGE


def test_oracle_totals_encode_exactly(xs):
    """The oracle's exact integer sums (units of 2^-1074) of the paper's
    dataset families, written as canonical states, encode to their value."""
    for kind in ("positive", "mixed", "anderson", "zero_sum"):
        for delta in (10, 2000):
            bits = workloads.family(kind, 20_000, delta, seed=delta)
            total = oracle.exact_sum(bits, "f64").total
            enc = xs.xsum_state_encode(state_bytes(canonical_digits(total)))
            assert read_encoding(enc) == (0, total)
            if total == 0:
                assert len(enc) == 12


def test_malformed_encodings_are_rejected(xs):
    good = xs.xsum_state_encode(state_bytes(canonical_digits(-(7 << 300) - 1)))
    bad = [
        b"",
        good[:11],
        b"XSS2" + good[4:],                             # magic
        good[:-1],                                      # length
        good + b"\0\0\0\0",
        good[:4] + struct.pack("<I", 8) + good[8:],     # special bits
        good[:8] + b"\x02" + good[9:],                  # sign
        good[:11] + b"\x01" + good[12:],                # reserved byte
        good[:9] + bytes([69]) + good[10:],             # run past the end
        good[:12] + bytes(4) + good[16:],               # run starts with zero
        struct.pack("<IIBBBB", 0x31535358, 0, 1, 0, 0, 0),   # negative zero
    ]
    for b in bad:
        with pytest.raises(xs.XsumError):
            xs.xsum_state_decode(b)
    # beyond the range: a digit at index 69
    big = struct.pack("<IIBBBB", 0x31535358, 0, 0, 69, 1, 0) + struct.pack("<I", 1)
    with pytest.raises(xs.XsumError) as e:
        xs.xsum_state_decode(big)
    assert e.value.status == xs.ERANGE


def test_encode_argument_checks(xs):
    with pytest.raises(xs.XsumError):
        xs.xsum_state_encode(state_bytes([0] * 67 + [0], special=8))
    with pytest.raises(xs.XsumError) as e:
        xs.xsum_state_encode(state_bytes([(1 << 62) + 1] + [0] * 67))
    assert e.value.status == xs.ERANGE
