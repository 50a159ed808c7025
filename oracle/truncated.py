"""Section 4's condition-number-sensitive summation, written out on the CPU:
r-truncated sparse superaccumulators summed up a balanced binary tree, a
stopping test at the root, and r <- r^2 until the test passes or nothing was
truncated.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Representation (Section 2).  A sparse superaccumulator is a map from
component index i to an integer mantissa Y_i; its value is sum Y_i R^i in
units of 2^-1074.  The radix is R = 2^32 and mantissas are integers (the
paper allows integer components in place of floating-point ones); every
mantissa lies in [-(R-1), R-1] ((alpha, beta)-regularised with
alpha = beta = R - 1).  The map holds the active indices: those that are
non-zero or were non-zero in an operand of the addition that produced it.

Addition (Section 2's lemma on regularised sums, used on sparse operands as
Section 2 and Lemma 3 describe): P_i = Y_i + Z_i over the union of the active
indices; a signed carry C_(i+1) in {-1, 0, 1} leaves W_i = P_i - C_(i+1) R in
[-(R-2), R-2]; S_i = W_i + C_i.  No carry moves further than one component.

Truncation (end of Section 2): the r-truncated form keeps the r most
significant active entries.  Everything it drops lies below the lowest kept
index k and is a sum of regularised mantissas, so its magnitude is below R^k.

The iteration (Section 4): start with r = 2; sum the leaves bottom-up,
truncating every partial sum to r entries; stop if the root passes the
stopping test, else set r <- r^2 and repeat; stop too once a pass truncated
nothing (its root is exact).

The stopping test.  The library returns the round-to-nearest-even result, so
the test used here certifies that rounding, not only a faithful one: with S
the root's value and B the sum, over every truncation on the tree, of R^k for
that truncation's lowest kept index k, the exact sum lies in [S - B, S + B];
if both ends round to the same value v and v lies outside that interval, the
exact sum rounds to v as well (rounding to nearest is monotone) and is not
equal to it (the inexact flag is set).  Otherwise the pass is not certified.

The paper's two tests are given too (``paper_tests``): y is unchanged by
adding and by subtracting n copies of the smallest value of the root's lowest
component, or the last place of y lies at least ceil(log2 n) bits above that
component.  They certify a faithful rounding.  Their argument needs every
truncated part to lie below the root's lowest kept component; the
active-index rule gives that: a node's kept indices stay active in every
node above it, so the root's r-th highest active index is at or above every
inner node's lowest kept index.  The test suite checks that whenever either
test passes, the root's rounding is faithful.
"""

from .ieee import decode, fmt_of, round_to_format
from .exact import ExactSum, finish, _as_bits

R_BITS = 32
R = 1 << R_BITS


def leaf(bits, fmt):
    """Sparse superaccumulator of one finite input: the integer
    (-1)^s m 2^q (units of 2^-1074) split into base-R mantissas that all
    carry the sign; zero components are not active.  None for NaN and
    infinities."""
    kind, s, m, q = decode(bits, fmt)
    if kind != "finite":
        return None
    v = m << q
    comps = {}
    i = 0
    while v:
        d = v & (R - 1)
        if d:
            comps[i] = -d if s else d
        v >>= R_BITS
        i += 1
    return comps


def carry_add(y, z):
    """Sum of two regularised sparse superaccumulators with one signed carry
    per component (the lemma on regularised sums in Section 2)."""
    p = {}
    for i in set(y) | set(z):
        p[i] = y.get(i, 0) + z.get(i, 0)
    s = {}
    for i, pi in p.items():
        c = 1 if pi >= R - 1 else (-1 if pi <= -(R - 1) else 0)
        s[i] = s.get(i, 0) + pi - c * R
        if c:
            s[i + 1] = s.get(i + 1, 0) + c
    return s


def value(y):
    return sum(v << (R_BITS * i) for i, v in y.items())


def truncate(y, r):
    """The r most significant active entries and the bound on what was
    dropped: R^k for k the lowest kept index when a non-zero entry was
    dropped, else 0."""
    idx = sorted(y, reverse=True)
    if len(idx) <= r:
        return dict(y), 0
    kept = {i: y[i] for i in idx[:r]}
    lost = any(y[i] for i in idx[r:])
    return kept, (1 << (R_BITS * idx[r - 1])) if lost else 0


def tree_sum(leaves, r):
    """Bottom-up pairwise summation of the leaves over a balanced binary tree
    (level by level, an odd node passing up unchanged), truncating every
    partial sum to r entries.  Returns (root, bound) with bound the sum of
    the cuts of every truncation (0 when nothing was lost)."""
    level = [(dict(lf), 0) for lf in leaves]
    if not level:
        return {}, 0
    while len(level) > 1:
        nxt = []
        for a in range(0, len(level) - 1, 2):
            (y, by), (z, bz) = level[a], level[a + 1]
            s, b = truncate(carry_add(y, z), r)
            nxt.append((s, by + bz + b))
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


def bits_value(bits, fmt):
    """Exact value of a finite bit pattern in units of 2^-1074 (None for an
    infinity or NaN)."""
    kind, s, m, q = decode(bits, fmt_of(fmt))
    if kind != "finite":
        return None
    return -(m << q) if s else (m << q)


def certified(total, bound, out_fmt):
    """The stopping test: (bits, flags) of the round-to-nearest-even result
    when every value in [total - bound, total + bound] rounds to it and it is
    not in that interval; the exact rounding when bound is 0; else None."""
    if bound == 0:
        return tuple(round_to_format(total, out_fmt))
    lo, hi = total - bound, total + bound
    blo, flo = round_to_format(lo, out_fmt)
    bhi, fhi = round_to_format(hi, out_fmt)
    if blo != bhi:
        return None
    v = bits_value(blo, out_fmt)
    if v is not None and lo <= v <= hi:
        return None
    return blo, flo | fhi


def paper_tests(root, n, out_fmt):
    """The paper's two stopping tests on a root (Section 4), as printed:
    (y unchanged by +-n eps_min, last place of y at least ceil(log2 n) bits
    above the lowest component's unit), where y is the root's value rounded
    to out_fmt and eps_min = R^(lowest active index)."""
    f = fmt_of(out_fmt)
    total = value(root)
    if not root:
        return True, True
    low = min(root)
    y, _ = round_to_format(total, out_fmt)
    yv = bits_value(y, out_fmt)
    if yv is None:
        return True, True
    eps = n << (R_BITS * low)
    t1 = round_to_format(yv + eps, out_fmt)[0] == y == round_to_format(yv - eps, out_fmt)[0]
    if yv == 0:
        return t1, False
    top = abs(yv).bit_length() - 1
    lsb = max(top - (f.precision - 1), f.qmin)
    logn = (n - 1).bit_length()
    return t1, lsb >= R_BITS * low + logn


def adaptive_sum(x, fmt, out_fmt=None, r0=2):
    """Section 4's iteration with the stopping test above.  Returns
    ((bits, flags), passes, r) with passes the number of tree passes and r
    the truncation parameter of the last one."""
    f = fmt_of(fmt)
    if out_fmt is None:
        out_fmt = "f32" if f.name == "bf16" else f.name
    leaves, specials = [], ExactSum()
    for b in _as_bits(x, f).tolist():
        lf = leaf(b, f)
        if lf is not None:
            leaves.append(lf)
            continue
        kind, s, _, _ = decode(b, f)
        if kind == "nan":
            specials.nan = True
        elif s:
            specials.ninf = True
        else:
            specials.pinf = True
    if specials.nan or specials.pinf or specials.ninf:
        # the result is decided by the special values alone
        return tuple(finish(specials, out_fmt)), 0, r0
    r, passes = r0, 0
    while True:
        passes += 1
        root, bound = tree_sum(leaves, r)
        total = value(root)
        res = certified(total, bound, out_fmt)
        if res is not None:
            return res, passes, r
        r = r * r
