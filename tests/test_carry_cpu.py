"""The carry-normalisation scheme the kernels use, checked exhaustively at a
small radix against plain integer arithmetic (Section 3, step 6: signed carry
propagation as a parallel prefix over a lookup table indexed by the incoming
carry).  The scheme is restated here from its description with radix 2^k in
place of 2^32; nothing is imported from the library.

Claims pinned:
  * two local carry steps take digits with |d| < 2^(2k-2) (the kernels'
    2^62 for k = 32) first into [-2^(k-2), 2^k + 2^(k-2)), then into
    [-1, 2^k], the top digit absorbing the carries;
  * on such digits, each digit's outgoing carry is a function of its incoming
    carry {-1, 0, 1} -> {-1, 0, 1}; composing these functions from the lowest
    digit up (in any grouping, as a parallel prefix does) gives every digit
    its carry-in, and the result is the canonical form of the same integer:
    digits in [0, 2^k) and a signed top digit.
No GPU."""

import itertools
import random

import pytest


def value(digits, radix):
    return sum(d * radix ** j for j, d in enumerate(digits))


def local_carry_step(digits, k):
    """One step: every digit keeps its low k bits and passes floor(d / 2^k)
    up; the top digit keeps everything."""
    radix = 1 << k
    out = list(digits)
    carries = [d >> k for d in digits]          # floor division
    for j in range(len(digits) - 1):
        out[j] = digits[j] & (radix - 1)
    for j in range(1, len(digits)):
        out[j] += carries[j - 1]
    return out


def transfer(d, radix):
    """Outgoing carry of digit d for incoming carry c = -1, 0, 1."""
    return tuple((d + c) // radix for c in (-1, 0, 1))


def compose(outer, inner):
    """outer after inner, both as tuples indexed by carry + 1."""
    return tuple(outer[inner[i] + 1] for i in range(3))


def prefix_normalise(digits, k, tree=False):
    """Carry-ins from an exclusive prefix of transfer functions (combined one
    after another, or by doubling as a wave does when tree is set), then one
    local fix-up."""
    radix = 1 << k
    fns = [transfer(d, radix) for d in digits[:-1]]
    n = len(fns)
    incl = list(fns)
    if not tree:
        for j in range(1, n):
            incl[j] = compose(fns[j], incl[j - 1])
    else:
        # Hillis-Steele doubling, as a wave does it: after the pass with
        # stride s, incl[j] covers digits max(0, j - 2s + 1) .. j
        s = 1
        while s < n:
            nxt = list(incl)
            for j in range(s, n):
                nxt[j] = compose(incl[j], incl[j - s])
            incl = nxt
            s *= 2
    cin = [0] + [incl[j][1] for j in range(n)]     # apply to carry 0
    out = [(digits[j] + cin[j]) % radix for j in range(n)]
    out.append(digits[-1] + cin[n])
    return out


def canonical(v, radix, length):
    digits = []
    for _ in range(length - 1):
        digits.append(v % radix)
        v //= radix
    digits.append(v)
    return digits


@pytest.mark.parametrize("k", [2, 3])
def test_two_local_steps_bound_the_digits(k):
    radix = 1 << k
    lim = 1 << (2 * k - 2)
    for digits in itertools.product(range(-lim + 1, lim), repeat=3):
        digits = list(digits) + [0]
        one = local_carry_step(digits, k)
        assert all(-(1 << (k - 2)) <= d < radix + (1 << (k - 2)) for d in one[:-1]), digits
        two = local_carry_step(one, k)
        assert all(-1 <= d <= radix for d in two[:-1]), digits
        assert value(two, radix) == value(digits, radix)


@pytest.mark.parametrize("k", [1, 2])
def test_transfer_functions_stay_in_minus_one_zero_one(k):
    radix = 1 << k
    for d in range(-1, radix + 1):
        assert set(transfer(d, radix)) <= {-1, 0, 1}


@pytest.mark.parametrize("k,length", [(1, 7), (2, 6)])
def test_prefix_gives_canonical_digits_exhaustively(k, length):
    radix = 1 << k
    for low in itertools.product(range(-1, radix + 1), repeat=length - 1):
        for top in (-2, -1, 0, 1):
            digits = list(low) + [top]
            got = prefix_normalise(digits, k)
            assert got == canonical(value(digits, radix), radix, length), digits


def test_prefix_in_tree_order_and_from_wide_digits():
    """Random wide digits: two local steps, then a doubling prefix, give the
    canonical digits of the same integer."""
    rng = random.Random(5)
    k = 5
    radix = 1 << k
    lim = 1 << (2 * k - 2)
    for _ in range(3000):
        length = rng.randrange(2, 40)
        digits = [rng.randrange(-lim + 1, lim) for _ in range(length - 1)] + [rng.randrange(-3, 4)]
        two = local_carry_step(local_carry_step(digits, k), k)
        got = prefix_normalise(two, k, tree=True)
        assert got == canonical(value(digits, radix), radix, length)
