// Device-side building blocks shared by the exact-sum kernels (gfx950).
//
// Representation (Section 2 of Goodrich & Eldawy, integer form of the
// regularised superaccumulator): the exact sum is kept as XSUM_DIGITS signed
// 64-bit digits of radix 2^32; digit j weighs 2^(32 j) in units of 2^-1074,
// the smallest binary64 subnormal, so every input of every supported format is
// an integer on this grid.  A digit is wider than its radix, so many chunks can
// be added into it before any carry has to move: the paper's lazy carry
// accumulation, which the overlap between neighbouring components allows.
//
// In the hot loop each lane adds into a private column of partial digits in
// LDS with fire-and-forget ds_add_u64 (no carries, no conflicts: lane l of
// digit d sits at word d*64 + l, so the 64 lanes always hit distinct banks).
//   binary64: value = (-1)^s m 2^p (units 2^-1074), m = M + [E>0] 2^52,
//             p = max(E,1) - 1.  With k = p >> 5, r = p & 31 the signed
//             T = +-m 2^r (|T| < 2^85) is added as two chunks: c0 = T mod 2^32
//             into digit k and c1 = floor(T / 2^32) (|c1| < 2^52) into digit
//             k+1.  A digit thus absorbs about 2^10 chunks before it must be
//             carried, so every lane carry-normalises its own column every
//             few hundred elements (cheap, LDS-local, sequential per lane).
//   binary32: the column is indexed by byte position and sign instead:
//             p = max(E,1) + 924, bin b = p >> 3, r = p & 7; the magnitude
//             m 2^r < 2^31 is added as one chunk to entry 2b (positive inputs)
//             or 2b + 1 (negative inputs) of the bin, which weighs 2^(8b).
//             Unsigned 64-bit entries absorb 2^33 chunks, so no normalisation
//             is needed, and keeping the sign in the entry index spares the
//             negation and the sign extension of every chunk.
//   bfloat16: as binary32 with the 8-bit significand: p = max(E,1) + 940,
//             magnitude m 2^r < 2^15.  Two elements (one 32-bit word) are
//             decoded at once with packed 16-bit integer operations.
// Infinities and NaNs (all-ones exponent) take the finite path like any other
// bit pattern; every lane tracks the largest exponent field (binary64) or
// magnitude (the binned formats) it saw, and after each tile the rare lanes
// that saw an all-ones exponent record the special value and add it again
// with the opposite sign, which cancels its contribution exactly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xsum.h"
#include "xsum_internal.h"

namespace xsum {

static constexpr int kDigits = XSUM_DIGITS;
static constexpr uint64_t kLow32 = 0xffffffffull;

// 16-byte vector as a native vector type (non-temporal loads need one).
typedef uint32_t vec4u __attribute__((ext_vector_type(4)));

template <int FMT> struct Geo;
// binary64: chunks reach digits 0..64; digit 65 is the column's carry top.
template <> struct Geo<XSUM_F64> {
    static constexpr int kN = 66;          // column entries per lane
    static constexpr int kPerVec = 2, kBytes = 8;
    static constexpr uint32_t kSpecFrom = 0x7ffu;   // tracked: exponent field
    static constexpr bool kBinned = false;
};
// binary32 / bfloat16: 33 byte-position bins (p >> 3 in [115, 147] and
// [117, 149]), two entries each: 2b for positive and 2b + 1 for negative
// magnitudes.
template <> struct Geo<XSUM_F32> {
    static constexpr int kN = 66;
    static constexpr int kPerVec = 4, kBytes = 4;
    static constexpr uint32_t kSpecFrom = 0x7f800000u;   // tracked: magnitude bits
    static constexpr bool kBinned = true;
    static constexpr int kBins = 33;
    static constexpr int kBin0 = 115;      // byte position of bin 0
};
template <> struct Geo<XSUM_BF16> {
    static constexpr int kN = 66;
    static constexpr int kPerVec = 8, kBytes = 2;
    static constexpr uint32_t kSpecFrom = 0x7f80u;       // tracked: magnitude bits
    static constexpr bool kBinned = true;
    static constexpr int kBins = 33;
    static constexpr int kBin0 = 117;
};

__device__ __forceinline__ void lds_add(uint64_t *p, uint64_t v)
{
    // The result is unused, so this is a no-return ds_add_u64.
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The same for a 32-bit entry (ds_add_u32).
__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint64_t lds_load(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_load(uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void wave_lds_fence()
{
    // every LDS operation of this wave issued so far has completed and is
    // ordered before what follows (other lanes' column entries are read
    // next).  The fence names LDS only, so loads and atomics in flight to
    // global memory are not waited for.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
}

// Special-value bits of a state: bit 0 NaN, bit 1 +inf, bit 2 -inf.
__device__ __forceinline__ uint32_t special_bits(bool mant_nonzero, bool neg)
{
    return mant_nonzero ? 1u : (neg ? 4u : 2u);
}

// One binary64 element (lo, hi words) into the lane's column (col points at
// the lane's entry of digit 0; digit d is col[d * 64]).
__device__ __forceinline__ void add_f64(uint32_t lo, uint32_t hi,
                                        uint64_t *col, uint32_t &emax)
{
    const uint32_t e = (hi >> 20) & 0x7ffu;
    emax = max(emax, e);
    const uint32_t p = max(e, 1u) - 1u;
    const uint32_t mhi = (hi & 0xfffffu) | (min(e, 1u) << 20);
    const int64_t m = (int64_t)(((uint64_t)mhi << 32) | lo);
    const int64_t sm = (int64_t)((int32_t)hi >> 31);     // 0 or -1
    const int64_t v = (m ^ sm) - sm;                     // signed significand
    const uint32_t r = p & 31u;
    const uint32_t c0 = (uint32_t)v << r;                // T mod 2^32
    const int64_t c1 = v >> (32 - r);                    // floor(T / 2^32)
    uint64_t *d = col + (p >> 5) * 64;
    lds_add(d, (uint64_t)c0);
    lds_add(d + 64, (uint64_t)c1);
}

// One binary32 element into the lane's column; amax keeps the largest
// magnitude bits seen (an all-ones exponent field makes it 0x7f800000 or more).
__device__ __forceinline__ void add_f32(uint32_t b, uint64_t *col,
                                        uint32_t &amax)
{
    const uint32_t a = b & 0x7fffffffu;
    amax = max(amax, a);
    // bits 23 and up: q = max(E,1) + 4 = p - 8*115, p = max(E,1) + 924
    const uint32_t u = max(a, 0x00800000u) + (4u << 23);
    // significand with its hidden bit (min(a, 2^23) is 2^23 exactly when E > 0)
    const uint32_t m = (a & 0x7fffffu) | min(a, 0x00800000u);
    const uint32_t t = m << ((u >> 23) & 7u);   // < 2^31
    // entry 2 (q >> 3) + sign: the bin index and the sign bit side by side
    const uint32_t idx = __builtin_amdgcn_alignbit(u >> 26, b, 31);
    lds_add(col + idx * 64, (uint64_t)t);
}

// Two bfloat16 elements (the halves of w) into the lane's column; amax keeps
// the largest magnitude bits seen in each half.  The column's entries are
// 64-bit, or 32-bit (C = uint32_t) in the single-sum kernel, which then
// flushes them before 2^17 chunks can reach one entry.
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

template <typename C>
__device__ __forceinline__ void add_bf16_pair(uint32_t w, C *col, u16x2 &amax)
{
    const u16x2 h = __builtin_bit_cast(u16x2, w);
    const u16x2 a = h & (u16x2)0x7fffu;
    amax = __builtin_elementwise_max(amax, a);
    // bits 7 to 15: q = max(E,1) + 4 = p - 8*117, p = max(E,1) + 940
    const u16x2 u = __builtin_elementwise_max(a, (u16x2)0x80u) + (u16x2)0x200u;
    const u16x2 m = (a & (u16x2)0x7fu) | __builtin_elementwise_min(a, (u16x2)0x80u);
    const u16x2 t = m << ((u >> (u16x2)7) & (u16x2)7);   // < 2^15
    // byte offset of entry 2 (q >> 3) + sign: q >> 3 sits in bits 10 to 15
    // of u.  64-bit entries are 512 bytes apart (sign to bit 9), 32-bit ones
    // 256 bytes (everything one bit lower)
    const uint32_t uu = __builtin_bit_cast(uint32_t, u);
    const uint32_t off = sizeof(C) == 8
                             ? (uu & 0xfc00fc00u) | ((w >> 6) & 0x02000200u)
                             : ((uu >> 1) & 0x7e007e00u) | ((w >> 7) & 0x01000100u);
    char *base = (char *)col;
    lds_add((C *)(base + (off & 0xffffu)), (C)t.x);
    lds_add((C *)(base + (off >> 16)), (C)t.y);
}

template <int FMT, typename C>
__device__ __forceinline__ void add_vec(const vec4u &q, C *col, uint32_t &emax)
{
    if constexpr (FMT == XSUM_F64) {
        add_f64(q.x, q.y, col, emax);
        add_f64(q.z, q.w, col, emax);
    } else if constexpr (FMT == XSUM_F32) {
        add_f32(q.x, col, emax);
        add_f32(q.y, col, emax);
        add_f32(q.z, col, emax);
        add_f32(q.w, col, emax);
    } else {
        u16x2 em = __builtin_bit_cast(u16x2, emax);
        add_bf16_pair(q.x, col, em);
        add_bf16_pair(q.y, col, em);
        add_bf16_pair(q.z, col, em);
        add_bf16_pair(q.w, col, em);
        emax = __builtin_bit_cast(uint32_t, em);
    }
}

// Special-value fix-up of one element already added by the fast path: if its
// exponent field is all ones, record it and add its negation.
__device__ __forceinline__ void fix_f64(uint32_t lo, uint32_t hi,
                                        uint64_t *col, uint32_t &spec)
{
    if (((hi >> 20) & 0x7ffu) == 0x7ffu) {
        spec |= special_bits(((hi & 0xfffffu) | lo) != 0, (hi >> 31) != 0);
        uint32_t dummy = 0;
        add_f64(lo, hi ^ 0x80000000u, col, dummy);
    }
}

__device__ __forceinline__ void fix_f32(uint32_t b, uint64_t *col,
                                        uint32_t &spec)
{
    if (((b >> 23) & 0xffu) == 0xffu) {
        spec |= special_bits((b & 0x7fffffu) != 0, (b >> 31) != 0);
        uint32_t dummy = 0;
        add_f32(b ^ 0x80000000u, col, dummy);
    }
}

// The same for the two bfloat16 halves of w: the special halves are added
// again with the opposite sign, the others are replaced by +0 (which adds 0).
template <typename C>
__device__ __forceinline__ void fix_bf16_pair(uint32_t w, C *col, uint32_t &spec)
{
    uint32_t neg = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint32_t hk = (w >> (16 * k)) & 0xffffu;
        if (((hk >> 7) & 0xffu) == 0xffu) {
            spec |= special_bits((hk & 0x7fu) != 0, (hk >> 15) != 0);
            neg |= (hk ^ 0x8000u) << (16 * k);
        }
    }
    if (neg) {
        u16x2 dummy = (u16x2)0;
        add_bf16_pair(neg, col, dummy);
    }
}

template <int FMT, typename C>
__device__ __forceinline__ void fix_vec(const vec4u &q, C *col, uint32_t &spec)
{
    if constexpr (FMT == XSUM_F64) {
        fix_f64(q.x, q.y, col, spec);
        fix_f64(q.z, q.w, col, spec);
    } else if constexpr (FMT == XSUM_F32) {
        fix_f32(q.x, col, spec);
        fix_f32(q.y, col, spec);
        fix_f32(q.z, col, spec);
        fix_f32(q.w, col, spec);
    } else {
        fix_bf16_pair(q.x, col, spec);
        fix_bf16_pair(q.y, col, spec);
        fix_bf16_pair(q.z, col, spec);
        fix_bf16_pair(q.w, col, spec);
    }
}

// Add U vectors, then fix up the (rare) lanes that met a special value.
template <int FMT, int U, typename C>
__device__ __forceinline__ void add_tile(const vec4u (&q)[U], C *col, uint32_t &spec)
{
    uint32_t emax = 0;      // largest exponent field (binary64) or magnitude
#pragma unroll
    for (int j = 0; j < U; ++j)
        add_vec<FMT>(q[j], col, emax);
    if constexpr (FMT == XSUM_BF16)     // two 16-bit fields
        emax = max(emax & 0xffffu, emax >> 16);
    if (__builtin_expect(emax >= Geo<FMT>::kSpecFrom, 0)) {
#pragma unroll
        for (int j = 0; j < U; ++j)
            fix_vec<FMT>(q[j], col, spec);
    }
}

// One element read with a scalar load (unaligned head, ragged tail).
template <int FMT, typename C>
__device__ __forceinline__ void add_scalar(const uint8_t *p, C *col, uint32_t &spec)
{
    uint32_t emax = 0;
    if constexpr (FMT == XSUM_F64) {
        const uint32_t *w = (const uint32_t *)p;
        add_f64(w[0], w[1], col, emax);
        fix_f64(w[0], w[1], col, spec);
    } else if constexpr (FMT == XSUM_F32) {
        const uint32_t b = *(const uint32_t *)p;
        add_f32(b, col, emax);
        fix_f32(b, col, spec);
    } else {
        const uint32_t w = *(const uint16_t *)p;    // upper half +0, adds 0
        u16x2 em = (u16x2)0;
        add_bf16_pair(w, col, em);
        fix_bf16_pair(w, col, spec);
    }
}

// Carry-normalise the lane's binary64 column in place: digits 0..kN-2 end in
// [0, 2^32), the last entry takes the carry.  The value is unchanged.
template <int N>
__device__ __forceinline__ void normalise_column(uint64_t *col)
{
    int64_t v[N];
#pragma unroll
    for (int d = 0; d < N; ++d)
        v[d] = (int64_t)lds_load(col + d * 64);
    int64_t carry = 0;
#pragma unroll
    for (int d = 0; d < N - 1; ++d) {
        const int64_t x = v[d] + carry;
        v[d] = (int64_t)((uint64_t)x & kLow32);
        carry = x >> 32;
    }
    v[N - 1] += carry;
#pragma unroll
    for (int d = 0; d < N; ++d)
        lds_store(col + d * 64, (uint64_t)v[d]);
}

// Add lo + hi 2^32 (lo in [0, 2^38), |hi| < 2^37) times the weight of column
// row d to the block's digit vector blk with LDS atomics.  A binary64 row is
// digit d itself; a binned row 2b + s is bin b (weight 2^(8(kBin0 + b))),
// negated for s = 1, moved onto its radix-2^32 digit by a byte shift.
template <int FMT>
__device__ __forceinline__ void add_row(int64_t *blk, int d, uint64_t lo, int64_t hi)
{
    using G = Geo<FMT>;
    int digit, shift;
    bool neg = false;
    if constexpr (G::kBinned) {
        const int bin = G::kBin0 + (d >> 1);
        digit = bin >> 2;
        shift = 8 * (bin & 3);
        neg = (d & 1) != 0;
    } else {
        digit = d;
        shift = 0;
    }
    // each shifted term stays below 2^62
    const uint64_t ls = lo << shift;
    const int64_t hs = (int64_t)((uint64_t)hi << shift);
    int64_t parts[3] = {(int64_t)(ls & kLow32),
                        (int64_t)(ls >> 32) + (int64_t)((uint64_t)hs & kLow32), hs >> 32};
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (parts[i])
            __hip_atomic_fetch_add(&blk[digit + i], neg ? -parts[i] : parts[i],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Block merge of one wave's columns.  Lane l takes column row l: it sums that
// row over the wave's 64 lanes, reading lane (c + l) mod 64 so the 64 lanes
// hit distinct banks.  Each entry splits as lo + hi 2^32 (lo in [0, 2^32))
// before summing so nothing can overflow; the sums go to the block's digit
// vector.  Rows 64 and 65 only receive chunks of inputs of magnitude 2^994
// and above in binary64 (and their carries), and of 2^125 and above in the
// binned formats, so instead of a second pass each lane adds its own two top
// entries, and only when one of them is non-zero anywhere in the wave.
template <int FMT, typename C>
__device__ __forceinline__ void merge_wave_columns(C (*cols)[64], int64_t *blk, int lane)
{
    using G = Geo<FMT>;
    static_assert(G::kN == 66, "two rows above the lanes");
    {
        const C *row = cols[lane];
        uint64_t lo = 0;
        int64_t hi = 0;
#pragma unroll 16
        for (int c = 0; c < 64; ++c) {
            const uint64_t val = row[(c + lane) & 63];
            lo += val & kLow32;
            hi += (int64_t)val >> 32;
        }
        add_row<FMT>(blk, lane, lo, hi);
    }
    uint64_t top[2];
    bool any = false;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        top[r] = cols[64 + r][lane];
        any |= top[r] != 0;
    }
    if (__ballot(any)) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if (top[r])
                add_row<FMT>(blk, 64 + r, top[r] & kLow32, (int64_t)top[r] >> 32);
    }
}

// ------------------------------------------------------- normalise + round --

// Carry transfer function of one digit f in [-1, 2^32]: for an incoming
// signed carry c in {-1, 0, 1} the outgoing carry is floor((f + c) / 2^32),
// again in {-1, 0, 1}.  Stored as three 2-bit fields: field c+1 holds
// carry+1.  (Section 3, step 6: signed carry propagation as a parallel prefix
// over a lookup table indexed by the incoming carry.)
__device__ __forceinline__ uint32_t carry_fn(int64_t f)
{
    uint32_t r = 0;
#pragma unroll
    for (int c = -1; c <= 1; ++c)
        r |= (uint32_t)(((f + c) >> 32) + 1) << (2 * (c + 1));
    return r;
}

// outer(inner(c)).
__device__ __forceinline__ uint32_t compose(uint32_t outer, uint32_t inner)
{
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint32_t j = (inner >> (2 * i)) & 3u;
        r |= ((outer >> (2 * j)) & 3u) << (2 * i);
    }
    return r;
}

__device__ __forceinline__ int apply_fn(uint32_t fn, int c)
{
    return (int)((fn >> (2 * (c + 1))) & 3u) - 1;
}

static constexpr uint32_t kIdentityFn = 0x24u;  // fields (0,1,2) -> (0,1,2)

// Wave-wide carry normalisation.  Lane l (l <= 33) holds digits 2l (a) and
// 2l+1 (b); lane 33's b is the signed top digit; lanes above 33 hold zeros.
// Inputs may be any int64 with |digit| < 2^62.  On return digits 0..66 are in
// [0, 2^32) and the top digit holds the rest, so the value is unchanged.
static __device__ __forceinline__ void normalise_wave(int64_t &a, int64_t &b, int lane)
{
    const bool top_lane = lane == 33;
    const bool live = lane <= 33;
    // two local carry steps: |d| < 2^62 -> [-2^30, 2^32 + 2^30) -> [-1, 2^32]
#pragma unroll
    for (int step = 0; step < 2; ++step) {
        const int64_t ca = a >> 32, cb = b >> 32;
        int64_t cin = __shfl_up(cb, 1, 64);
        if (lane == 0)
            cin = 0;
        a = (int64_t)((uint64_t)a & kLow32) + cin;
        b = top_lane ? b + ca : (int64_t)((uint64_t)b & kLow32) + ca;
        if (!live) {
            a = 0;
            b = 0;
        }
    }
    // exclusive prefix (lowest digit first) of the per-lane transfer
    // functions, Hillis-Steele over the wave
    const uint32_t fa = carry_fn(a);
    const uint32_t fb = top_lane ? kIdentityFn : carry_fn(b);
    uint32_t x = compose(fb, fa);
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint32_t y = __shfl_up(x, s, 64);
        if (lane >= s)
            x = compose(x, y);
    }
    uint32_t excl = __shfl_up(x, 1, 64);
    if (lane == 0)
        excl = kIdentityFn;
    const int cin_a = apply_fn(excl, 0);
    const int cin_b = apply_fn(fa, cin_a);
    a = (int64_t)((uint64_t)(a + cin_a) & kLow32);
    b = top_lane ? b + cin_b : (int64_t)((uint64_t)(b + cin_b) & kLow32);
    if (!live) {
        a = 0;
        b = 0;
    }
}

struct OutFormat {
    int width;      // bits
    int t;          // stored mantissa bits
    int prec;       // t + 1
    int qmin;       // exponent of the smallest subnormal, units of 2^-1074
    uint32_t emax;  // all-ones exponent field
};

__device__ __forceinline__ OutFormat out_format(int fmt)
{
    if (fmt == XSUM_F64)
        return OutFormat{64, 52, 53, 0, 0x7ffu};
    if (fmt == XSUM_F32)
        return OutFormat{32, 23, 24, 925, 0xffu};
    return OutFormat{16, 7, 8, 941, 0xffu};
}

__device__ __forceinline__ uint64_t fmt_inf(const OutFormat &f, bool neg)
{
    return ((uint64_t)neg << (f.width - 1)) | ((uint64_t)f.emax << f.t);
}

__device__ __forceinline__ uint64_t fmt_qnan(const OutFormat &f)
{
    return ((uint64_t)f.emax << f.t) | (1ull << (f.t - 1));
}

// Round-to-nearest-even of the magnitude whose top non-zero digit is h
// (value w2), with the next two digits w1, w0 (zero below digit 0) and a
// sticky flag for any non-zero digit below h-2.
static __device__ __forceinline__ uint64_t round_magnitude(bool neg, int h, uint32_t w2, uint32_t w1,
                                    uint32_t w0, bool sticky_below,
                                    const OutFormat &f, uint32_t &flags)
{
    typedef unsigned __int128 u128;
    const u128 W = ((u128)w2 << 64) | ((u128)w1 << 32) | (u128)w0;
    const int base = 32 * (h - 2);                  // grid exponent of W's bit 0
    const int B = 32 * h + 31 - __builtin_clz(w2);  // leading one
    int q = max(B - (f.prec - 1), f.qmin);          // exponent of the last place
    const int s = q - base;                         // >= 12 by construction
    u128 mant;
    bool rbit, sticky;
    if (s >= 128) {
        mant = 0;
        rbit = false;
        sticky = true;
    } else {
        mant = W >> s;
        rbit = ((W >> (s - 1)) & 1) != 0;
        sticky = sticky_below || (W & ((((u128)1) << (s - 1)) - 1)) != 0;
    }
    if (rbit || sticky)
        flags |= XSUM_FLAG_INEXACT;
    if (rbit && (sticky || (mant & 1)))
        mant += 1;
    if (mant == ((u128)1 << f.prec)) {
        mant >>= 1;
        q += 1;
    }
    uint64_t efield, mfield;
    const uint64_t m64 = (uint64_t)mant;
    if (m64 < (1ull << (f.prec - 1))) {
        efield = 0;                                 // subnormal (q == qmin)
        mfield = m64;
    } else {
        efield = (uint64_t)(q - f.qmin + 1);
        mfield = m64 - (1ull << (f.prec - 1));
    }
    if (efield >= f.emax) {
        flags |= XSUM_FLAG_OVERFLOW | XSUM_FLAG_INEXACT;
        return fmt_inf(f, neg);
    }
    return ((uint64_t)neg << (f.width - 1)) | (efield << f.t) | mfield;
}

__device__ __forceinline__ uint64_t low_mask(int k)
{
    return k <= 0 ? 0ull : (k >= 64 ? ~0ull : ((1ull << k) - 1));
}

// Round canonical digits (output of normalise_wave) held by the wave.
// Returns the bit pattern in every lane.
// Result decided by special inputs (IEEE addition): any NaN, or +inf with
// -inf, gives the quiet NaN; otherwise an infinity gives that infinity.
// Returns false when no special value was seen.
__device__ __forceinline__ bool special_result(uint32_t special,
                                               const OutFormat &f,
                                               uint64_t &bits, uint32_t &flags)
{
    if ((special & 1u) || ((special & 6u) == 6u)) {
        flags = XSUM_FLAG_NAN | ((special & 6u) ? XSUM_FLAG_INF : 0u);
        bits = fmt_qnan(f);
        return true;
    }
    if (special & 6u) {
        flags = XSUM_FLAG_INF;
        bits = fmt_inf(f, (special & 4u) != 0);
        return true;
    }
    return false;
}

static __device__ __forceinline__ uint64_t round_wave(int64_t a, int64_t b, int lane,
                               uint32_t special, int out_fmt, uint32_t &flags)
{
    const OutFormat f = out_format(out_fmt);
    flags = 0;
    uint64_t sbits;
    if (special_result(special, f, sbits, flags))
        return sbits;
    const int64_t top = __shfl(b, 33, 64);
    const bool neg = top < 0;
    const bool is_digit_b = lane < 33;  // lane 33's b is the top digit
    uint64_t ua = (uint64_t)a, ub = is_digit_b ? (uint64_t)b : 0ull;
    bool range_error = !(top == 0 || top == -1);
    if (neg) {
        // |S| = 2^(32*67) - sum u_j 2^(32 j): two's complement of digits 0..66
        const uint64_t nza = __ballot(ua != 0), nzb = __ballot(ub != 0);
        const int za = nza ? 2 * __builtin_ctzll(nza) : 1 << 20;
        const int zb = nzb ? 2 * __builtin_ctzll(nzb) + 1 : 1 << 20;
        const int z = min(za, zb);
        if (z >= (1 << 20))
            range_error = true;
        const int ja = 2 * lane, jb = 2 * lane + 1;
        ua = ja < z ? 0 : (ja == z ? (1ull << 32) - ua : kLow32 - ua);
        ub = jb < z ? 0 : (jb == z ? (1ull << 32) - ub : kLow32 - ub);
        if (lane > 33)
            ua = 0;
        if (!is_digit_b)
            ub = 0;
    }
    if (range_error) {
        // beyond 2^(32*67 - 1074): far above every format's range
        flags = XSUM_FLAG_OVERFLOW | XSUM_FLAG_INEXACT;
        return fmt_inf(f, neg);
    }
    const uint64_t ma = __ballot(ua != 0), mb = __ballot(ub != 0);
    if (!ma && !mb)
        return 0;                                   // exact zero -> +0
    const int ha = ma ? 2 * (63 - __builtin_clzll(ma)) : -1;
    const int hb = mb ? 2 * (63 - __builtin_clzll(mb)) + 1 : -1;
    const int h = max(ha, hb);
    uint32_t w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = h - i;
        const int src = j >= 0 ? (j >> 1) : 0;
        const uint64_t va = __shfl(ua, src, 64), vb = __shfl(ub, src, 64);
        w[i] = j < 0 ? 0u : (uint32_t)((j & 1) ? vb : va);
    }
    const int lim = h - 2;  // digits strictly below h-2 feed the sticky bit
    const bool sticky = ((ma & low_mask((lim + 1) >> 1)) |
                         (mb & low_mask(lim >> 1))) != 0;
    return round_magnitude(neg, h, w[0], w[1], w[2], sticky, f, flags);
}

__device__ __forceinline__ void store_result(void *out, int out_fmt,
                                             uint64_t bits)
{
    if (out_fmt == XSUM_F64)
        *(uint64_t *)out = bits;
    else if (out_fmt == XSUM_F32)
        *(uint32_t *)out = (uint32_t)bits;
    else
        *(uint16_t *)out = (uint16_t)bits;
}

// Last-block work of an accumulation launch, run by one full wave.  SYS: the
// state was filled with system-scope atomics by other waves of this launch,
// so every access here is system-scope too.  Otherwise the state comes from
// earlier launches and agent scope suffices.
template <bool SYS>
static __device__ __forceinline__ void finish_state(xsum_acc_t *acc, const Finish &fin, int lane)
{
    constexpr int kScope = SYS ? __HIP_MEMORY_SCOPE_SYSTEM : __HIP_MEMORY_SCOPE_AGENT;
    int64_t a = 0, b = 0;
    const bool live = lane <= 33;
    if (fin.mode == kRound) {       // take the digits and leave zeros
        if (live) {
            a = __hip_atomic_exchange(&acc->digit[2 * lane], (int64_t)0, __ATOMIC_RELAXED, kScope);
            b = __hip_atomic_exchange(&acc->digit[2 * lane + 1], (int64_t)0, __ATOMIC_RELAXED,
                                      kScope);
        }
    } else if (live) {
        a = __hip_atomic_load(&acc->digit[2 * lane], __ATOMIC_RELAXED, kScope);
        b = __hip_atomic_load(&acc->digit[2 * lane + 1], __ATOMIC_RELAXED, kScope);
    }
    const uint32_t special = __hip_atomic_load(&acc->special, __ATOMIC_RELAXED, kScope);
    normalise_wave(a, b, lane);
    if (fin.mode == kRound) {
        uint32_t flags;
        const uint64_t bits = round_wave(a, b, lane, special, fin.out_fmt, flags);
        if (lane == 0) {
            if (fin.out_slot8)
                *(uint64_t *)fin.out = bits;
            else
                store_result(fin.out, fin.out_fmt, bits);
            if (fin.flags)
                *fin.flags = flags;
            __hip_atomic_store(&acc->special, 0u, __ATOMIC_RELAXED, kScope);
            __hip_atomic_store(&acc->ticket, 0u, __ATOMIC_RELAXED, kScope);
        }
    } else {
        if (live) {
            __hip_atomic_store(&acc->digit[2 * lane], a, __ATOMIC_RELAXED, kScope);
            __hip_atomic_store(&acc->digit[2 * lane + 1], b, __ATOMIC_RELAXED, kScope);
        }
        if (lane == 0)
            __hip_atomic_store(&acc->ticket, 0u, __ATOMIC_RELAXED, kScope);
    }
}

}  // namespace xsum
