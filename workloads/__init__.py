"""Seeded synthetic inputs, as IEEE bit patterns.

This module only builds inputs; it holds none of the summation method's
arithmetic and imports neither the oracle nor the library.  Both the tests
(oracle side and GPU side) and the benchmark draw their inputs from here.

Every generator is deterministic in its seed.  Large arrays are produced in
chunks of CHUNK elements, chunk i drawing from the i-th child of
``numpy.random.SeedSequence(seed)``, so the result does not depend on how many
threads generate it.

Workloads (shapes follow the paper's experiments, Section 6, and the
benchmark configurations of this library):

* ``config1``: n = 10^6 doubles, random sign, uniform 52-bit mantissa,
  exponent uniform in [-50, 50].
* ``config2``: n = 2^28 doubles, ill-conditioned by construction: 2^27 values
  a_i (exponent uniform in [-1000, 1000]) and their exact negations, 1% of the
  negations replaced by perturbations p_j (exponent uniform in [-1074, -900]),
  seeded shuffle.  The exact sum is sum_j (a_j + p_j) over the replaced pairs.
* ``config3``: n = 2^31 doubles z * 2^k, z ~ N(0,1), k uniform in [-500, 500];
  one entry in every 1000 is replaced by a subnormal or by +-DBL_MAX (the
  +-DBL_MAX entries have exactly balanced signs).
* ``config4``: segmented batch, 10^6 segments with lognormal lengths (median
  256, sigma 2 in natural-log units, clipped to [1, 2^20]) and a per-segment
  dtype mix of 50% binary64, 37.5% binary32, 12.5% bfloat16; values as in
  config 1; every segment starts on a 16-byte boundary.
* ``serving_trace``: Poisson arrivals, log-uniform request sizes, binary64 or
  binary32 requests with values shaped like config 2.
* The four dataset families of the paper's experiments (positive, mixed sign,
  Anderson's ill-conditioned, zero sum) with an exponent range delta.
* ``set_equality``: the reduction from set equality used in the paper's lower
  bound (Section 3): -2^(tau*c_i) and +2^(tau*d_i) sum to zero exactly when the
  multisets C and D are equal.
* ``crafted_cases``: boundary and carry-path cases.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 24

F64, F32, BF16 = "f64", "f32", "bf16"
DTYPE_CODE = {F64: 0, F32: 1, BF16: 2}
ITEMSIZE = {F64: 8, F32: 4, BF16: 2}
UINT = {F64: np.uint64, F32: np.uint32, BF16: np.uint16}

DBL_MAX_BITS = 0x7FEFFFFFFFFFFFFF
FLT_MAX_BITS = 0x7F7FFFFF


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def _chunked(n, seed, fill, dtype=np.uint64):
    """out[i*CHUNK:(i+1)*CHUNK] = fill(rng_i, count), rng_i from child i."""
    out = np.empty(n, dtype=dtype)
    nchunks = (n + CHUNK - 1) // CHUNK
    children = np.random.SeedSequence(seed).spawn(max(nchunks, 1))

    def work(i):
        lo = i * CHUNK
        hi = min(n, lo + CHUNK)
        out[lo:hi] = fill(np.random.default_rng(children[i]), hi - lo)

    if nchunks <= 1:
        if n:
            work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


# ---------------------------------------------------------------- building --

def f64_normal(sign, k, mant):
    """Bit patterns of (-1)^sign * (1 + mant/2^52) * 2^k for k in [-1022, 1023]."""
    sign = np.asarray(sign, dtype=np.uint64)
    e = (np.asarray(k, dtype=np.int64) + 1023).astype(np.uint64)
    return (sign << np.uint64(63)) | (e << np.uint64(52)) | \
        np.asarray(mant, dtype=np.uint64)


def f32_normal(sign, k, mant):
    """Bit patterns of (-1)^sign * (1 + mant/2^23) * 2^k for k in [-126, 127]."""
    sign = np.asarray(sign, dtype=np.uint32)
    e = (np.asarray(k, dtype=np.int64) + 127).astype(np.uint32)
    return (sign << np.uint32(31)) | (e << np.uint32(23)) | \
        np.asarray(mant, dtype=np.uint32)


def bf16_normal(sign, k, mant):
    """Bit patterns of (-1)^sign * (1 + mant/2^7) * 2^k for k in [-126, 127]."""
    sign = np.asarray(sign, dtype=np.uint16)
    e = (np.asarray(k, dtype=np.int64) + 127).astype(np.uint16)
    return (sign << np.uint16(15)) | (e << np.uint16(7)) | \
        np.asarray(mant, dtype=np.uint16)


def uniform_values(rng, count, fmt, kmin, kmax):
    """Random sign, uniform mantissa field, exponent uniform in [kmin, kmax]."""
    s = rng.integers(0, 2, size=count)
    k = rng.integers(kmin, kmax + 1, size=count)
    if fmt == F64:
        return f64_normal(s, k, rng.integers(0, 1 << 52, size=count, dtype=np.uint64))
    if fmt == F32:
        return f32_normal(s, k, rng.integers(0, 1 << 23, size=count, dtype=np.uint32))
    return bf16_normal(s, k, rng.integers(0, 1 << 7, size=count, dtype=np.uint16))


def f64_with_leading_bit(rng, count, kmin, kmax):
    """Random sign, leading bit at 2^k with k uniform in [kmin, kmax], uniform
    bits below it.  For k < -1022 the value is a subnormal whose leading bit is
    2^k (the remaining bits below it are uniform)."""
    s = rng.integers(0, 2, size=count).astype(np.uint64)
    k = rng.integers(kmin, kmax + 1, size=count)
    mant = rng.integers(0, 1 << 52, size=count, dtype=np.uint64)
    normal = k >= -1022
    bits = np.where(normal, f64_normal(s, np.where(normal, k, 0), mant), 0)
    sub = ~normal
    if np.any(sub):
        width = (k[sub] + 1074).astype(np.uint64)           # 0 .. 51
        lead = np.uint64(1) << width
        low = mant[sub] & (lead - np.uint64(1))
        bits[sub] = (s[sub] << np.uint64(63)) | lead | low
    return bits.astype(np.uint64)


def f32_with_leading_bit(rng, count, kmin, kmax):
    """binary32 analogue of ``f64_with_leading_bit`` (subnormal below -126)."""
    s = rng.integers(0, 2, size=count).astype(np.uint32)
    k = rng.integers(kmin, kmax + 1, size=count)
    mant = rng.integers(0, 1 << 23, size=count, dtype=np.uint32)
    normal = k >= -126
    bits = np.where(normal, f32_normal(s, np.where(normal, k, 0), mant), 0)
    sub = ~normal
    if np.any(sub):
        width = (k[sub] + 149).astype(np.uint32)
        lead = np.uint32(1) << width
        low = mant[sub] & (lead - np.uint32(1))
        bits[sub] = (s[sub] << np.uint32(31)) | lead | low
    return bits.astype(np.uint32)


def _shuffle_in_place(a, seed):
    np.random.default_rng(np.random.SeedSequence([seed, 0x5EED])).shuffle(a)


# ----------------------------------------------------------------- configs --

def config1(n=1_000_000, seed=0):
    """binary64, random sign, uniform mantissa, exponent uniform in [-50, 50]."""
    return _chunked(n, seed, lambda r, c: uniform_values(r, c, F64, -50, 50))


def config2(log2n=28, seed=0, variant="a", pert_fraction=0.01):
    """Cancelling pairs plus perturbations (see the module docstring).

    Returns (bits, terms): bits is the shuffled input of n = 2^log2n values;
    terms holds the values whose exact sum equals the exact sum of bits:
    a_j and p_j for every replaced pair j (variant "a", one negation replaced)
    or the two perturbations of every replaced pair (variant "b", both members
    replaced).
    """
    half = 1 << (log2n - 1)
    a = _chunked(half, seed, lambda r, c: uniform_values(r, c, F64, -1000, 1000))
    neg = a ^ np.uint64(1 << 63)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    nrep = int(pert_fraction * half)
    idx = np.sort(rng.choice(half, size=nrep, replace=False))
    pert = f64_with_leading_bit(rng, nrep, -1074, -900)
    neg[idx] = pert
    if variant == "a":
        terms = np.concatenate([a[idx], pert])
    elif variant == "b":
        pert2 = f64_with_leading_bit(rng, nrep, -1074, -900)
        a[idx] = pert2
        terms = np.concatenate([pert2, pert])
    else:
        raise ValueError(variant)
    bits = np.concatenate([a, neg])
    del a, neg
    _shuffle_in_place(bits, seed)
    return bits, terms


def config3_specials(n, seed):
    """Positions and bit patterns of config 3's special entries.

    One entry per block of 1000 (block b covers [1000 b, 1000 b + 1000)) at a
    seeded offset.  The first half of a seeded label order are subnormals
    (random sign, uniform non-zero mantissa); the rest are +-DBL_MAX with
    exactly as many + as - (an odd count leaves one subnormal extra)."""
    nspec = n // 1000
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    pos = np.arange(nspec, dtype=np.int64) * 1000 + \
        rng.integers(0, 1000, size=nspec)
    nsub = nspec // 2
    nmax = nspec - nsub
    if nmax % 2:
        nsub += 1
        nmax -= 1
    vals = np.empty(nspec, dtype=np.uint64)
    sub_s = rng.integers(0, 2, size=nsub).astype(np.uint64)
    sub_m = rng.integers(1, 1 << 52, size=nsub, dtype=np.uint64)
    vals[:nsub] = (sub_s << np.uint64(63)) | sub_m
    max_s = np.repeat(np.array([0, 1], dtype=np.uint64), nmax // 2)
    vals[nsub:] = (max_s << np.uint64(63)) | np.uint64(DBL_MAX_BITS)
    order = rng.permutation(nspec)
    return pos, vals[order]


def config3(n=1 << 31, seed=0, balanced=True):
    """binary64 z * 2^k, z ~ N(0,1), k uniform in [-500, 500], with one
    special entry per 1000 (see ``config3_specials``).  balanced=False gives
    the +-DBL_MAX entries independent random signs (the sum overflows)."""
    def fill(r, c):
        z = r.standard_normal(c)
        k = r.integers(-500, 501, size=c)
        return np.ldexp(z, k).view(np.uint64)

    bits = _chunked(n, seed, fill)
    pos, vals = config3_specials(n, seed)
    if not balanced:
        rng = np.random.default_rng(np.random.SeedSequence([seed, 33]))
        ismax = (vals & np.uint64(0x7FFFFFFFFFFFFFFF)) == np.uint64(DBL_MAX_BITS)
        s = rng.integers(0, 2, size=int(ismax.sum())).astype(np.uint64)
        vals[ismax] = (s << np.uint64(63)) | np.uint64(DBL_MAX_BITS)
    bits[pos] = vals
    return bits


def segment_lengths(nseg, seed, median=256.0, sigma=2.0, lmax=1 << 20):
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    L = np.rint(rng.lognormal(np.log(median), sigma, size=nseg))
    return np.clip(L, 1, lmax).astype(np.int64)


def segment_dtypes(nseg, seed):
    """Per-segment dtype code: U < 0.5 binary64, U < 0.875 binary32, else
    bfloat16 (so a quarter of the 32-bit segments are bfloat16)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 5]))
    u = rng.random(nseg)
    return np.where(u < 0.5, 0, np.where(u < 0.875, 1, 2)).astype(np.uint32)


def config4(nseg=1_000_000, seed=0, lengths=None, dtypes=None, kmin=-50,
            kmax=50, align=16):
    """Segmented batch.  Returns (buf, desc): buf is a uint8 array holding
    every segment, each starting at a multiple of ``align`` bytes; desc is a
    structured array of (byte_offset u64, length u64, dtype u32, reserved
    u32), dtype codes 0 binary64, 1 binary32, 2 bfloat16."""
    L = segment_lengths(nseg, seed) if lengths is None else \
        np.asarray(lengths, dtype=np.int64)
    D = segment_dtypes(nseg, seed) if dtypes is None else \
        np.asarray(dtypes, dtype=np.uint32)
    nseg = len(L)
    size = L * np.array([8, 4, 2], dtype=np.int64)[D]
    padded = (size + align - 1) // align * align
    offs = np.zeros(nseg, dtype=np.int64)
    if nseg:
        offs[1:] = np.cumsum(padded)[:-1]
    total = int(padded.sum()) if nseg else 0
    buf = np.zeros(total, dtype=np.uint8)
    desc = np.zeros(nseg, dtype=SEGMENT_DTYPE)
    desc["byte_offset"] = offs
    desc["length"] = L
    desc["dtype"] = D
    children = np.random.SeedSequence([seed, 6]).spawn(max(1, (nseg + 4095) // 4096))
    names = [F64, F32, BF16]

    def work(ci):
        # values of one chunk of 4096 segments are drawn per format in bulk,
        # then cut into the chunk's segments in order
        rng = np.random.default_rng(children[ci])
        lo, hi = ci * 4096, min(nseg, (ci + 1) * 4096)
        pools, taken = [], [0, 0, 0]
        for d in range(3):
            cnt = int(L[lo:hi][D[lo:hi] == d].sum())
            pools.append(uniform_values(rng, cnt, names[d], kmin, kmax).astype(UINT[names[d]])
                         .view(np.uint8))
        for s in range(lo, hi):
            d = int(D[s])
            nb = int(L[s]) * ITEMSIZE[names[d]]
            o = int(offs[s])
            buf[o:o + nb] = pools[d][taken[d]:taken[d] + nb]
            taken[d] += nb

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(len(children))))
    return buf, desc


SEGMENT_DTYPE = np.dtype([("byte_offset", "<u8"), ("length", "<u8"),
                          ("dtype", "<u4"), ("reserved", "<u4")])


def serving_trace(seed=0, rate=2000.0, duration=60.0, smin=1e3, smax=1e8):
    """Request arrivals: (arrival_time_s, size, dtype_code) arrays.

    Poisson arrivals at ``rate`` per second over ``duration`` seconds,
    size log-uniform in [smin, smax], dtype binary64 or binary32 with equal
    probability."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.5) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration]
    m = len(t)
    size = np.exp(rng.uniform(np.log(smin), np.log(smax), size=m)).astype(np.int64)
    dt = rng.integers(0, 2, size=m).astype(np.uint32)
    return t, size, dt


def serving_payload(size, fmt, seed):
    """Values shaped like config 2 for one request: cancelling pairs, 1% of
    the negations replaced by tiny perturbations, shuffled.  binary32
    requests use exponents in [-120, 120] and perturbations in [-149, -127].
    An odd size ends with one extra perturbation."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 8]))
    half = size // 2
    if fmt == F64:
        a = uniform_values(rng, half, F64, -1000, 1000)
        neg = a ^ np.uint64(1 << 63)
        pert = lambda c: f64_with_leading_bit(rng, c, -1074, -900)
    else:
        a = uniform_values(rng, half, F32, -120, 120)
        neg = a ^ np.uint32(1 << 31)
        pert = lambda c: f32_with_leading_bit(rng, c, -149, -127)
    nrep = int(0.01 * half)
    if nrep:
        idx = rng.choice(half, size=nrep, replace=False)
        neg[idx] = pert(nrep)
    parts = [a, neg]
    if size % 2:
        parts.append(pert(1))
    bits = np.concatenate(parts)
    rng.shuffle(bits)
    return bits


# ---------------------------------------------------- experiment families --

def family(kind, n, delta, seed=0, fmt=F64):
    """The four dataset families of the paper's experiments (Section 6).

    kind: "positive", "mixed", "anderson" or "zero_sum"; exponents are
    uniform in [-delta/2, delta/2].  "anderson" subtracts the (floating-point)
    mean of a mixed-sign set from every element; "zero_sum" is a shuffled set
    of values and their negations (exact sum zero)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 9, delta]))
    lo, hi = -(delta // 2), delta - delta // 2
    if kind == "zero_sum":
        h = n // 2
        a = uniform_values(rng, h, fmt, lo, hi)
        bits = np.concatenate([a, a ^ UINT[fmt](1 << (8 * ITEMSIZE[fmt] - 1))])
        if n % 2:
            bits = np.concatenate([bits, np.zeros(1, dtype=UINT[fmt])])
        rng.shuffle(bits)
        return bits
    bits = uniform_values(rng, n, fmt, lo, hi)
    if kind == "positive":
        return bits & UINT[fmt]((1 << (8 * ITEMSIZE[fmt] - 1)) - 1)
    if kind == "mixed":
        return bits
    if kind == "anderson":
        if fmt != F64:
            raise ValueError("anderson family is generated in binary64")
        x = bits.view(np.float64)
        with np.errstate(over="ignore", invalid="ignore"):
            mean = np.mean(x)
            y = x - mean
        return y.view(np.uint64)
    raise ValueError(kind)


def set_equality(C, D, n_hint=None):
    """binary64 patterns of -2^(tau*c) for c in C and +2^(tau*d) for d in D,
    tau the smallest power of two above log2(|C|+|D|) (Section 3, lower
    bound).  Exponents must stay in the normal range."""
    n = n_hint or (len(C) + len(D))
    tau = 1
    while tau <= np.log2(max(n, 2)):
        tau *= 2
    ec = np.asarray(C, dtype=np.int64) * tau
    ed = np.asarray(D, dtype=np.int64) * tau
    if len(ec) and (ec.min() < -1022 or ec.max() > 1023):
        raise ValueError("exponent out of range")
    if len(ed) and (ed.min() < -1022 or ed.max() > 1023):
        raise ValueError("exponent out of range")
    neg = f64_normal(np.ones(len(ec), dtype=np.uint64), ec, np.zeros(len(ec), dtype=np.uint64))
    pos = f64_normal(np.zeros(len(ed), dtype=np.uint64), ed, np.zeros(len(ed), dtype=np.uint64))
    return np.concatenate([neg, pos]).astype(np.uint64), tau


# ---------------------------------------------------------- crafted cases --

def _d(*vals):
    return np.array(vals, dtype=np.float64).view(np.uint64)


def crafted_cases():
    """(name, fmt, bits) triples covering boundaries, rounding ties, overflow
    thresholds, subnormal results, special values and long carry/borrow
    chains."""
    tiny = 5e-324
    dmax = np.finfo(np.float64).max
    two = lambda k: float(np.ldexp(1.0, k))
    cases = [
        ("empty", F64, np.zeros(0, dtype=np.uint64)),
        ("pos_zero", F64, _d(0.0)),
        ("neg_zero", F64, _d(-0.0)),
        ("neg_zeros", F64, _d(-0.0, -0.0, -0.0)),
        ("one", F64, _d(1.0)),
        ("min_subnormal", F64, _d(tiny)),
        ("max_subnormal", F64, np.array([0x000FFFFFFFFFFFFF], dtype=np.uint64)),
        ("min_normal_from_subnormals", F64,
         np.array([0x0008000000000000, 0x0008000000000000], dtype=np.uint64)),
        ("subnormal_sum", F64, _d(tiny, tiny, tiny, -tiny * 2)),
        ("tie_to_even_down", F64, _d(1.0, two(-53))),
        ("tie_to_even_up", F64, _d(1.0, 3 * two(-53))),
        ("tie_broken_by_sticky", F64, _d(1.0, two(-53), tiny)),
        ("tie_broken_by_neg_sticky", F64, _d(1.0, two(-53), -tiny)),
        ("overflow_threshold", F64, _d(dmax, two(970))),
        ("below_overflow_threshold", F64, _d(dmax, two(970), -tiny)),
        ("neg_overflow", F64, _d(-dmax, -dmax)),
        ("dmax_cancel", F64, _d(dmax, dmax, -dmax, -dmax, 1.0)),
        ("big_minus_tiny", F64, _d(two(1023), -tiny)),
        ("tiny_minus_big", F64, _d(-two(1023), tiny)),
        ("borrow_chain", F64, _d(two(1023), -two(1023), tiny, -two(-1000))),
        ("carry_chain", F64, _d(*([dmax] * 8), *([-dmax] * 7), -two(971), tiny)),
        ("exact_cancel", F64, _d(1.5, -1.5, two(-1070), -two(-1070))),
        ("pinf", F64, _d(np.inf, 1.0)),
        ("ninf", F64, _d(-np.inf, 1.0, -3.0)),
        ("inf_minus_inf", F64, _d(np.inf, -np.inf)),
        ("nan", F64, np.array([0x7FF0000000000001, 0], dtype=np.uint64)),
        ("neg_nan", F64, np.array([0xFFF8000000000000, 0x3FF0000000000000], dtype=np.uint64)),
        ("f32_basic", F32, np.array([1.0, 2.0 ** -24, 2.0 ** -149], dtype=np.float32).view(np.uint32)),
        ("f32_overflow", F32, np.array([FLT_MAX_BITS, FLT_MAX_BITS], dtype=np.uint32)),
        ("f32_threshold", F32, np.array([FLT_MAX_BITS, 0x73000000], dtype=np.uint32)),
        ("f32_subnormal", F32, np.array([1, 1, 0x80000001, 0x007FFFFF], dtype=np.uint32)),
        ("f32_tie", F32, np.array([1.0, 2.0 ** -24], dtype=np.float32).view(np.uint32)),
        ("f32_cancel", F32, np.array([3.0, -3.0, -0.0], dtype=np.float32).view(np.uint32)),
        ("f32_specials", F32, np.array([0x7F800000, 0x3F800000], dtype=np.uint32)),
        ("bf16_basic", BF16, np.array([0x3F80, 0x3F80, 0x0001, 0x8001, 0x7F7F], dtype=np.uint16)),
        ("bf16_cancel", BF16, np.array([0x4040, 0xC040], dtype=np.uint16)),
        ("bf16_nan", BF16, np.array([0x7FC1, 0x3F80], dtype=np.uint16)),
    ]
    return cases
