"""The exact sum as a wide fixed-point integer, and its rounding.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 of the paper observes that summing every input as a fixed-point
number with enough bits on both sides of the binary point is error-free; with
the binary point shifted, that number is a plain integer.  ``exact_sum`` is
that definition written out with Python's unbounded ``int``: one addition per
input, no blocking, no reordering.  ``finish`` applies the Section 1
requirement (a faithful rounding) as round-to-nearest-even, plus the IEEE
rules for infinities and NaNs, which the paper does not discuss (it assumes
finite inputs).

``fraction_sum`` is an independent brute force through ``fractions.Fraction``
used only to pin the oracle on small inputs.
"""

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .ieee import (UNIT_EXP, FLAG_NAN, FLAG_INF, decode, fmt_of,
                   round_to_format)


@dataclass
class ExactSum:
    """Exact state of a sum: the finite part in units of 2^-1074 and which
    special values were seen."""
    total: int = 0
    nan: bool = False
    pinf: bool = False
    ninf: bool = False

    def merge(self, other):
        return ExactSum(self.total + other.total, self.nan or other.nan,
                        self.pinf or other.pinf, self.ninf or other.ninf)


def _as_bits(x, fmt):
    """Bit patterns of x as a 1-D numpy unsigned array of the format's width."""
    f = fmt_of(fmt)
    dt = {64: np.uint64, 32: np.uint32, 16: np.uint16}[f.width]
    a = np.asarray(x)
    if a.dtype != dt:
        a = a.view(dt)
    return a.reshape(-1)


def exact_sum(x, fmt):
    """Exact sum of the inputs x (floats or their bit patterns) of format fmt.

    Each finite input contributes (-1)^s * m * 2^q to one Python int, with
    (s, m, q) from ``ieee.decode``.  Specials only set flags.
    """
    f = fmt_of(fmt)
    acc = ExactSum()
    for b in _as_bits(x, f).tolist():
        kind, s, m, q = decode(b, f)
        if kind == "nan":
            acc.nan = True
        elif kind == "inf":
            if s:
                acc.ninf = True
            else:
                acc.pinf = True
        else:
            term = m << q
            acc.total += -term if s else term
    return acc


def finish(acc, out_fmt):
    """Round an exact state to out_fmt.  Returns (bits, flags).

    Special values decide first: any NaN, or both infinities, give the
    canonical quiet NaN; otherwise an infinity input gives that infinity.
    Only a sum of finite inputs is rounded, to nearest with ties to even;
    an exact zero gives +0.
    """
    f = fmt_of(out_fmt)
    if acc.nan or (acc.pinf and acc.ninf):
        flags = FLAG_NAN | (FLAG_INF if (acc.pinf or acc.ninf) else 0)
        return f.qnan, flags
    if acc.pinf:
        return f.pinf, FLAG_INF
    if acc.ninf:
        return f.ninf, FLAG_INF
    return round_to_format(acc.total, f)


def oracle_sum(x, fmt, out_fmt=None):
    """Correctly rounded (RNE) sum of x.  out_fmt defaults to fmt, except
    bfloat16 inputs, whose sum is returned as binary32."""
    f = fmt_of(fmt)
    if out_fmt is None:
        out_fmt = "f32" if f.name == "bf16" else f.name
    return finish(exact_sum(x, f), out_fmt)


def value_fraction(bits, fmt):
    """Exact rational value of a finite bit pattern (via ``ieee.decode``)."""
    kind, s, m, q = decode(bits, fmt)
    assert kind == "finite"
    v = Fraction(m) * Fraction(2) ** (q + UNIT_EXP)
    return -v if s else v


def fraction_sum(values):
    """Brute-force exact sum of Python floats through Fraction (pins only)."""
    return sum((Fraction(v) for v in values), Fraction(0))


def fraction_to_format(v, fmt):
    """Bit pattern of the RNE rounding of the rational v to fmt, through the
    exact integer grid: v must be a multiple of 2^-1074 (every sum of inputs
    is)."""
    scaled = v * Fraction(2) ** (-UNIT_EXP)
    assert scaled.denominator == 1
    return round_to_format(scaled.numerator, fmt)
