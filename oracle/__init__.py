"""CPU oracle for the exact sum of IEEE binary floating-point numbers.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import, call, link or execute anything
in this package.  The product path (the HIP library and its Python binding)
never touches it and shares no code with it.

What it computes (Goodrich & Eldawy, "Parallel Algorithms for Summing
Floating-Point Numbers"):

* Section 2 (first representation): every float is an integer multiple of the
  smallest subnormal, so the exact sum is a wide fixed-point number, i.e. a
  big integer with a shifted binary point.  Summing in it is exact.  The
  oracle keeps that integer as a Python ``int`` in units of 2^-1074
  (``exact.exact_sum``) or, for large inputs, as one 128-bit integer per
  biased exponent accumulated by a multithreaded C routine
  (``binned.exact_sum_binned``) and folded into the same Python ``int``.
* Section 1 (problem statement): the result must be a faithful rounding of
  the exact sum.  The oracle picks round-to-nearest, ties-to-even, which is one
  of the two faithful answers and is unique (``ieee.round_to_format``).

Nothing here follows the paper's parallel algorithms; the oracle is the plain
definition, written out.

Parity unpinned by the paper: the conventions it leaves open, which the
oracle fixes in ``exact.finish`` and ``ieee.round_to_format``: a finite sum
that rounds past the largest finite value gives an infinity with an overflow
flag; NaN and infinity inputs give what IEEE 754 addition gives; an exact zero
gives +0; the output format defaults to binary64 for binary64 input and
binary32 otherwise.  These are checked against IEEE 754 arithmetic (CPython
floats, numpy, torch) and for self-consistency, not against the paper.
"""

from .ieee import (FORMATS, UNIT_EXP, FLAG_INEXACT, FLAG_OVERFLOW, FLAG_NAN,
                   FLAG_INF, Format, decode, round_to_format, fmt_of)
from .exact import (ExactSum, exact_sum, finish, oracle_sum, fraction_sum,
                    fraction_to_format, value_fraction)
from .binned import (exact_sum_binned, oracle_sum_binned, build_binned,
                     segmented_exact_sums, segmented_oracle_sums)

__all__ = [
    "FORMATS", "UNIT_EXP", "FLAG_INEXACT", "FLAG_OVERFLOW", "FLAG_NAN",
    "FLAG_INF", "Format", "decode", "round_to_format", "fmt_of", "ExactSum",
    "exact_sum", "finish", "oracle_sum", "fraction_sum", "fraction_to_format",
    "value_fraction", "exact_sum_binned", "oracle_sum_binned", "build_binned",
    "segmented_exact_sums", "segmented_oracle_sums",
]
from . import truncated
from .truncated import adaptive_sum
