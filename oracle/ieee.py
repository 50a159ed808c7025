"""IEEE 754 binary formats on integers: decode a bit pattern, round an exact
integer sum to a bit pattern.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 1 and Section 2 of the paper describe a float as a triple (b, M, E)
with t mantissa bits and l exponent bits; double precision has t=52, l=11 and
single precision t=23, l=8.  The exponent bias in the paper's formula is
garbled; it is read here as the IEEE 754 bias 2^(l-1)-1, with E=0 encoding
subnormals (the paper does not assume normalised inputs) and E=2^l-1 encoding
infinities and NaNs.  bfloat16 (t=7, l=8) is the upper half of a binary32.

Every finite value of every format here is an integer multiple of 2^-1074, the
smallest double subnormal, so all exact sums are kept as Python ints in units
of 2^-1074 (UNIT_EXP).
"""

from dataclasses import dataclass

UNIT_EXP = -1074

# Result flags.  Their numeric values are part of the library's C interface
# convention; they are restated here, not imported.
FLAG_INEXACT = 1   # the returned finite value differs from the exact sum
FLAG_OVERFLOW = 2  # the exact finite sum rounds beyond the largest finite value
FLAG_NAN = 4       # the result is NaN (a NaN input, or +inf and -inf inputs)
FLAG_INF = 8       # at least one input was an infinity


@dataclass(frozen=True)
class Format:
    name: str
    t: int  # stored mantissa bits
    l: int  # exponent bits

    @property
    def bias(self):
        return (1 << (self.l - 1)) - 1

    @property
    def width(self):
        return 1 + self.l + self.t

    @property
    def emax_field(self):
        return (1 << self.l) - 1

    @property
    def precision(self):
        return self.t + 1

    @property
    def qmin(self):
        """Exponent of the smallest subnormal, in units of 2^UNIT_EXP."""
        return (1 - self.bias - self.t) - UNIT_EXP

    @property
    def qnan(self):
        """Canonical quiet NaN bit pattern (positive sign, top mantissa bit)."""
        return (self.emax_field << self.t) | (1 << (self.t - 1))

    @property
    def pinf(self):
        return self.emax_field << self.t

    @property
    def ninf(self):
        return (1 << (self.width - 1)) | self.pinf


FORMATS = {
    "f64": Format("f64", 52, 11),
    "f32": Format("f32", 23, 8),
    "bf16": Format("bf16", 7, 8),
}


def fmt_of(fmt):
    return fmt if isinstance(fmt, Format) else FORMATS[fmt]


def decode(bits, fmt):
    """Split a bit pattern into its IEEE meaning.

    Returns ("nan", sign, None, None), ("inf", sign, None, None) or
    ("finite", sign, m, q) with value = (-1)^sign * m * 2^(q + UNIT_EXP).
    For normal numbers m carries the implicit leading one (2^t + M) and
    q = E - bias - t - UNIT_EXP; subnormals (E = 0) have m = M and the
    exponent of E = 1.
    """
    f = fmt_of(fmt)
    bits = int(bits)
    sign = (bits >> (f.width - 1)) & 1
    e = (bits >> f.t) & f.emax_field
    mfield = bits & ((1 << f.t) - 1)
    if e == f.emax_field:
        return ("nan" if mfield else "inf", sign, None, None)
    if e == 0:
        m = mfield
        e_eff = 1
    else:
        m = (1 << f.t) | mfield
        e_eff = e
    q = (e_eff - f.bias - f.t) - UNIT_EXP
    return ("finite", sign, m, q)


def round_to_format(total, fmt):
    """Round the exact value total * 2^UNIT_EXP to the nearest value of
    format fmt, ties to even (IEEE 754 roundTiesToEven).

    Returns (bits, flags) with flags a combination of FLAG_INEXACT and
    FLAG_OVERFLOW.  An exact zero gives +0.  A magnitude that rounds past the
    largest finite value gives an infinity of the sum's sign.
    """
    f = fmt_of(fmt)
    total = int(total)
    if total == 0:
        return 0, 0
    sign = 1 if total < 0 else 0
    a = -total if sign else total
    p = f.precision
    top = a.bit_length() - 1          # position of the leading one
    q = max(top - (p - 1), f.qmin)    # exponent of the result's last place
    shift = q                         # a is in units of 2^0 of the grid
    flags = 0
    if shift <= 0:
        mant = a << (-shift)
        rem_nonzero = False
    else:
        mant = a >> shift
        rem = a - (mant << shift)
        half = 1 << (shift - 1)
        rem_nonzero = rem != 0
        if rem > half or (rem == half and (mant & 1)):
            mant += 1
    if rem_nonzero:
        flags |= FLAG_INEXACT
    if mant == (1 << p):              # rounding carried into a new binade
        mant >>= 1
        q += 1
    if mant < (1 << (p - 1)):         # subnormal (only possible at q == qmin)
        assert q == f.qmin
        efield = 0
        mfield = mant
    else:
        efield = q - f.qmin + 1
        mfield = mant - (1 << (p - 1))
    if efield >= f.emax_field:
        flags |= FLAG_OVERFLOW | FLAG_INEXACT
        return (f.ninf if sign else f.pinf), flags
    bits = (sign << (f.width - 1)) | (efield << f.t) | mfield
    return bits, flags
