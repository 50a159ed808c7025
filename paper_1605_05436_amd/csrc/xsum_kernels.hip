// HIP kernels for exact floating-point summation on gfx950 (CDNA4).
//
// Representation (Section 2 of Goodrich & Eldawy, integer form of the
// regularised superaccumulator): the exact sum is kept as XSUM_DIGITS signed
// 64-bit digits of radix 2^32; digit j weighs 2^(32 j) in units of 2^-1074,
// the smallest binary64 subnormal, so every input of every supported format is
// an integer on this grid.  A digit holds a 32-bit chunk plus 31 bits of
// headroom, so up to 2^31 chunks can be added into one digit before any carry
// has to move (the paper's lazy carry accumulation, which its one-bit overlap
// between components makes possible).
//
// Pipeline of one exact sum (Section 3 steps 2, 5, 6, 7; Section 5's scan
// algorithm, whose whole accumulator fits in fast memory; Section 6's
// combine / reduce / post-process structure):
//   1. load      128-bit non-temporal loads, grid-stride over 16-byte vectors
//   2. split     decode sign, exponent, significand; cut the significand,
//                shifted to its digit boundary, into 2 or 3 signed chunks
//   3. add       chunk j goes to digit k+j of the lane's private column in
//                LDS with a fire-and-forget ds_add_u64 (no carries)
//   4. block     the wave's 64 columns are summed per digit with one local
//                carry split; the block's digits go to the global state with
//                int64 atomics (one per non-zero digit)
//   5. ticket    the last block to finish takes over the global state
//   6. normalise two local carry steps bring every digit to [-1, 2^32]; a
//                wave-wide prefix over the carry transfer functions
//                {-1,0,1} -> {-1,0,1} (the paper's lookup-table prefix) gives
//                canonical digits and the sign
//   7. round     the top non-zero digit and its two neighbours plus a sticky
//                bit give the round-to-nearest-even result
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xsum.h"
#include "xsum_internal.h"

namespace xsum {

static constexpr int kDigits = XSUM_DIGITS;
static constexpr uint64_t kLow32 = 0xffffffffull;

// 16-byte vector as a native vector type (non-temporal loads need one).
typedef uint32_t vec4u __attribute__((ext_vector_type(4)));

// Digit window touched by each input format.
//   binary64: value = (-1)^s m 2^(p-1074), m = M + [E>0] 2^52, p = max(E,1)-1
//             p in [0, 2045] -> k = p>>5 in [0, 63], 3 chunks -> digits 0..65
//   binary32: m = M + [E>0] 2^23, p = max(E,1) + 924 in [925, 1178]
//             k in [28, 36], 2 chunks -> digits 28..37
//   bfloat16: the upper half of a binary32 (exact widening), as binary32
template <int FMT> struct Geo;
template <> struct Geo<XSUM_F64> {
    static constexpr int kLo = 0, kN = 66, kPerVec = 2, kBytes = 8;
};
template <> struct Geo<XSUM_F32> {
    static constexpr int kLo = 28, kN = 10, kPerVec = 4, kBytes = 4;
};
template <> struct Geo<XSUM_BF16> {
    static constexpr int kLo = 28, kN = 10, kPerVec = 8, kBytes = 2;
};

__device__ __forceinline__ void lds_add(uint64_t *p, uint64_t v)
{
    // Each column belongs to one lane, so the wavefront scope suffices; the
    // result is unused, so this is a no-return ds_add_u64.
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Special-value bits of the state: bit 0 NaN, bit 1 +inf, bit 2 -inf.
__device__ __forceinline__ uint32_t special_bits(bool mant_nonzero, bool neg)
{
    return mant_nonzero ? 1u : (neg ? 4u : 2u);
}

// One binary64 element (lo, hi words) into the lane's column.  col points at
// the lane's entry of digit kLo; digit d is at col[(d - kLo) * 64].
__device__ __forceinline__ void add_f64(uint32_t lo, uint32_t hi,
                                        uint64_t *col, uint32_t &spec)
{
    uint32_t e = (hi >> 20) & 0x7ffu;
    if (__builtin_expect(e == 0x7ffu, 0)) {
        spec |= special_bits(((hi & 0xfffffu) | lo) != 0, (hi >> 31) != 0);
        hi &= 0x80000000u;  // contributes a signed zero instead
        lo = 0;
        e = 0;
    }
    const uint32_t p = max(e, 1u) - 1u;
    const uint32_t mhi = (hi & 0xfffffu) | (min(e, 1u) << 20);
    const int64_t m = (int64_t)(((uint64_t)mhi << 32) | lo);
    const int64_t sm = (int64_t)((int32_t)hi >> 31);     // 0 or -1
    const int64_t v = (m ^ sm) - sm;                     // signed significand
    const uint32_t r = p & 31u;
    // T = v * 2^r, |T| < 2^85: T = c0 + c1 2^32 + c2 2^64 with c0, c1 in
    // [0, 2^32) and c2 = floor(T / 2^64) signed.
    const uint64_t low = (uint64_t)v << r;
    const int64_t c2 = (v >> 32) >> (32 - r);
    uint64_t *d = col + (p >> 5) * 64;
    lds_add(d, low & kLow32);
    lds_add(d + 64, low >> 32);
    lds_add(d + 128, (uint64_t)c2);
}

// One binary32 element (or a bfloat16 widened by a 16-bit shift).
__device__ __forceinline__ void add_f32(uint32_t b, uint64_t *col,
                                        uint32_t &spec)
{
    uint32_t e = (b >> 23) & 0xffu;
    if (__builtin_expect(e == 0xffu, 0)) {
        spec |= special_bits((b & 0x7fffffu) != 0, (b >> 31) != 0);
        b &= 0x80000000u;
        e = 0;
    }
    const uint32_t p = max(e, 1u) + 924u;
    const int32_t m = (int32_t)((b & 0x7fffffu) | (min(e, 1u) << 23));
    const int32_t sm = (int32_t)b >> 31;
    const int64_t v = (int64_t)((m ^ sm) - sm);
    // T = v * 2^r, |T| < 2^56: T = c0 + c1 2^32, c0 in [0, 2^32), c1 signed.
    const int64_t t = (int64_t)((uint64_t)v << (p & 31u));
    uint64_t *d = col + ((p >> 5) - 28) * 64;
    lds_add(d, (uint64_t)t & kLow32);
    lds_add(d + 64, (uint64_t)(t >> 32));
}

template <int FMT>
__device__ __forceinline__ void add_vec(const vec4u &q, uint64_t *col,
                                        uint32_t &spec)
{
    if constexpr (FMT == XSUM_F64) {
        add_f64(q.x, q.y, col, spec);
        add_f64(q.z, q.w, col, spec);
    } else if constexpr (FMT == XSUM_F32) {
        add_f32(q.x, col, spec);
        add_f32(q.y, col, spec);
        add_f32(q.z, col, spec);
        add_f32(q.w, col, spec);
    } else {
        add_f32(q.x << 16, col, spec);
        add_f32(q.x & 0xffff0000u, col, spec);
        add_f32(q.y << 16, col, spec);
        add_f32(q.y & 0xffff0000u, col, spec);
        add_f32(q.z << 16, col, spec);
        add_f32(q.z & 0xffff0000u, col, spec);
        add_f32(q.w << 16, col, spec);
        add_f32(q.w & 0xffff0000u, col, spec);
    }
}

template <int FMT>
__device__ __forceinline__ void add_scalar(const uint8_t *p, uint64_t *col,
                                           uint32_t &spec)
{
    if constexpr (FMT == XSUM_F64) {
        const uint32_t *w = (const uint32_t *)p;
        add_f64(w[0], w[1], col, spec);
    } else if constexpr (FMT == XSUM_F32) {
        add_f32(*(const uint32_t *)p, col, spec);
    } else {
        add_f32((uint32_t)(*(const uint16_t *)p) << 16, col, spec);
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
__device__ void normalise_wave(int64_t &a, int64_t &b, int lane)
{
    const bool top_lane = lane == 33;
    const bool live = lane <= 33;
    // two local carry steps: |d| < 2^62 -> (-2^30, 2^32 + 2^30) -> [-1, 2^32]
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
__device__ uint64_t round_magnitude(bool neg, int h, uint32_t w2, uint32_t w1,
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
__device__ uint64_t round_wave(int64_t a, int64_t b, int lane,
                               uint32_t special, int out_fmt, uint32_t &flags)
{
    const OutFormat f = out_format(out_fmt);
    flags = 0;
    if ((special & 1u) || ((special & 6u) == 6u)) {
        flags = XSUM_FLAG_NAN | ((special & 6u) ? XSUM_FLAG_INF : 0u);
        return fmt_qnan(f);
    }
    if (special & 6u) {
        flags = XSUM_FLAG_INF;
        return fmt_inf(f, (special & 4u) != 0);
    }
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

__device__ __forceinline__ int64_t gload(const int64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void gstore(int64_t *p, int64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-block work of an accumulation launch, run by one full wave.
__device__ void finish_state(xsum_acc_t *acc, const Finish &fin, int lane)
{
    int64_t a = 0, b = 0;
    const bool live = lane <= 33;
    uint32_t special;
    if (fin.mode == kRound) {
        if (live) {
            a = (int64_t)atomicExch((unsigned long long *)&acc->digit[2 * lane], 0ull);
            b = (int64_t)atomicExch((unsigned long long *)&acc->digit[2 * lane + 1], 0ull);
        }
        special = __hip_atomic_load(&acc->special, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    } else {
        if (live) {
            a = gload(&acc->digit[2 * lane]);
            b = gload(&acc->digit[2 * lane + 1]);
        }
        special = __hip_atomic_load(&acc->special, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    }
    normalise_wave(a, b, lane);
    if (fin.mode == kRound) {
        uint32_t flags;
        const uint64_t bits = round_wave(a, b, lane, special, fin.out_fmt, flags);
        if (lane == 0) {
            store_result(fin.out, fin.out_fmt, bits);
            if (fin.flags)
                *fin.flags = flags;
            __hip_atomic_store(&acc->special, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&acc->ticket, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
        if (live) {
            gstore(&acc->digit[2 * lane], a);
            gstore(&acc->digit[2 * lane + 1], b);
        }
        if (lane == 0)
            __hip_atomic_store(&acc->ticket, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------ accumulate --

// x: first element; head elements precede the 16-byte-aligned vector part
// of nvec 16-byte vectors, followed by tail elements.
template <int FMT, int WAVES, int U>
__global__ __launch_bounds__(WAVES * 64) void accumulate_kernel(
    const uint8_t *__restrict__ x, uint32_t head, uint64_t nvec,
    uint32_t tail, xsum_acc_t *acc, Finish fin)
{
    using G = Geo<FMT>;
    constexpr int kThreads = WAVES * 64;
    constexpr uint64_t kTile = (uint64_t)kThreads * U;  // vectors per block step
    __shared__ uint64_t cols[WAVES][G::kN][64];
    __shared__ int64_t blk[kDigits];
    __shared__ uint32_t blk_spec;
    __shared__ int is_last;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *col = &cols[wave][0][lane];
#pragma unroll
    for (int d = 0; d < G::kN; ++d)
        col[d * 64] = 0;
    if (tid < kDigits)
        blk[tid] = 0;
    if (tid == 0)
        blk_spec = 0;
    uint32_t spec = 0;

    const vec4u *v = (const vec4u *)(x + (uint64_t)head * G::kBytes);
    const uint64_t gstep = (uint64_t)gridDim.x * kTile;
    uint64_t tb = (uint64_t)blockIdx.x * kTile;

    // Full tiles, software-pipelined: the next tile's loads are in flight
    // while the current one is split and added.
    if (tb + kTile <= nvec) {
        vec4u qa[U], qb[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            qa[j] = __builtin_nontemporal_load(v + tb + j * kThreads + tid);
        for (;;) {
            uint64_t nb = tb + gstep;
            bool more = nb + kTile <= nvec;
            if (more) {
#pragma unroll
                for (int j = 0; j < U; ++j)
                    qb[j] = __builtin_nontemporal_load(v + nb + j * kThreads + tid);
            }
#pragma unroll
            for (int j = 0; j < U; ++j)
                add_vec<FMT>(qa[j], col, spec);
            tb = nb;
            if (!more)
                break;
            nb = tb + gstep;
            more = nb + kTile <= nvec;
            if (more) {
#pragma unroll
                for (int j = 0; j < U; ++j)
                    qa[j] = __builtin_nontemporal_load(v + nb + j * kThreads + tid);
            }
#pragma unroll
            for (int j = 0; j < U; ++j)
                add_vec<FMT>(qb[j], col, spec);
            tb = nb;
            if (!more)
                break;
        }
    }
    // At most one partial tile exists (the last); its owner finishes it.
    if (tb < nvec) {
        for (int j = 0; j < U; ++j) {
            const uint64_t i = tb + (uint64_t)j * kThreads + tid;
            if (i < nvec)
                add_vec<FMT>(__builtin_nontemporal_load(v + i), col, spec);
        }
    }
    // Unaligned head and ragged tail (fewer than 16 bytes each).
    if (blockIdx.x == 0) {
        if ((uint32_t)tid < head)
            add_scalar<FMT>(x + (uint64_t)tid * G::kBytes, col, spec);
        if ((uint32_t)tid < tail)
            add_scalar<FMT>(x + (uint64_t)head * G::kBytes + nvec * 16 +
                                (uint64_t)tid * G::kBytes,
                            col, spec);
    }
    __syncthreads();

    // Block merge: lane l sums digit l (and l+64) over the wave's 64 columns,
    // reading column (c + l) mod 64 so the 64 lanes hit distinct banks.  Each
    // column digit splits as lo + hi 2^32 (lo in [0, 2^32)); lo stays, hi
    // moves one digit up: this is the one local carry step of the merge.
    for (int d = lane; d < G::kN; d += 64) {
        const uint64_t *row = &cols[wave][d][0];
        uint64_t lo = 0;
        int64_t hi = 0;
#pragma unroll 16
        for (int c = 0; c < 64; ++c) {
            const uint64_t val = row[(c + lane) & 63];
            lo += val & kLow32;
            hi += (int64_t)val >> 32;
        }
        if (lo)
            __hip_atomic_fetch_add(&blk[G::kLo + d], (int64_t)lo,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (hi)
            __hip_atomic_fetch_add(&blk[G::kLo + d + 1], hi, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (spec)
        __hip_atomic_fetch_or(&blk_spec, spec, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();

    // Grid merge: add the block's non-zero digits into the global state.
    if (tid < kDigits) {
        const int64_t dv = blk[tid];
        if (dv)
            atomicAdd((unsigned long long *)&acc->digit[tid], (unsigned long long)dv);
    }
    if (tid == 0 && blk_spec)
        atomicOr(&acc->special, blk_spec);
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned t = atomicAdd(&acc->ticket, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last)
        return;
    __threadfence();
    if (wave == 0)
        finish_state(acc, fin, lane);
}

// --------------------------------------------------- small state kernels --

__global__ __launch_bounds__(64) void finalize_kernel(const xsum_acc_t *acc,
                                                      int out_fmt, void *out,
                                                      uint32_t *flags)
{
    const int lane = threadIdx.x;
    int64_t a = 0, b = 0;
    if (lane <= 33) {
        a = acc->digit[2 * lane];
        b = acc->digit[2 * lane + 1];
    }
    const uint32_t special = acc->special;
    normalise_wave(a, b, lane);
    uint32_t fl;
    const uint64_t bits = round_wave(a, b, lane, special, out_fmt, fl);
    if (lane == 0) {
        store_result(out, out_fmt, bits);
        if (flags)
            *flags = fl;
    }
}

__global__ __launch_bounds__(64) void merge_kernel(xsum_acc_t *dst,
                                                   const xsum_acc_t *src)
{
    const int lane = threadIdx.x;
    int64_t a = 0, b = 0;
    if (lane <= 33) {
        a = dst->digit[2 * lane] + src->digit[2 * lane];
        b = dst->digit[2 * lane + 1] + src->digit[2 * lane + 1];
    }
    normalise_wave(a, b, lane);
    if (lane <= 33) {
        dst->digit[2 * lane] = a;
        dst->digit[2 * lane + 1] = b;
    }
    if (lane == 0)
        dst->special |= src->special;
}

__global__ void zero_kernel(uint64_t *p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------------------------- launchers --

int element_size(int dtype)
{
    return dtype == XSUM_F64 ? 8 : dtype == XSUM_F32 ? 4 : 2;
}

// Single-sum launch shapes.  binary64 columns take 66 x 64 x 8 B = 33 KiB per
// wave, so a 4-wave block fills one CU's LDS (160 KiB); the narrow formats
// need 5 KiB per wave and run several blocks per CU.
static constexpr int kWaves = 4;
static constexpr int kUnroll = 8;

int persistent_blocks(int dtype, int cu_count)
{
    return dtype == XSUM_F64 ? cu_count : 4 * cu_count;
}

template <int FMT>
static hipError_t launch_fmt(const void *x, uint64_t n, xsum_acc_t *acc,
                             const Finish &fin, int cu_count,
                             const Shape &shape, hipStream_t stream)
{
    using G = Geo<FMT>;
    const uintptr_t addr = (uintptr_t)x;
    uint64_t head = ((16 - (addr & 15)) & 15) / G::kBytes;
    if (head > n)
        head = n;
    const uint64_t rest = n - head;
    const uint64_t nvec = rest / G::kPerVec;
    const uint64_t tail = rest - nvec * G::kPerVec;
    const uint64_t tile = (uint64_t)kWaves * 64 * kUnroll;
    const uint64_t tiles = (nvec + tile - 1) / tile;
    uint64_t blocks = shape.blocks > 0 ? (uint64_t)shape.blocks
                                       : (uint64_t)persistent_blocks(FMT, cu_count);
    if (blocks > tiles)
        blocks = tiles;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL((accumulate_kernel<FMT, kWaves, kUnroll>), dim3((unsigned)blocks),
                       dim3(kWaves * 64), 0, stream, (const uint8_t *)x,
                       (uint32_t)head, nvec, (uint32_t)tail, acc, fin);
    return hipGetLastError();
}

hipError_t launch_accumulate(const void *x, uint64_t n, int dtype,
                             xsum_acc_t *acc, const Finish &fin, int cu_count,
                             const Shape &shape, hipStream_t stream)
{
    switch (dtype) {
    case XSUM_F64:
        return launch_fmt<XSUM_F64>(x, n, acc, fin, cu_count, shape, stream);
    case XSUM_F32:
        return launch_fmt<XSUM_F32>(x, n, acc, fin, cu_count, shape, stream);
    default:
        return launch_fmt<XSUM_BF16>(x, n, acc, fin, cu_count, shape, stream);
    }
}

hipError_t launch_finalize(const xsum_acc_t *acc, int out_fmt, void *out,
                           uint32_t *flags, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, stream, acc,
                       out_fmt, out, flags);
    return hipGetLastError();
}

hipError_t launch_merge(xsum_acc_t *dst, const xsum_acc_t *src,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(merge_kernel, dim3(1), dim3(64), 0, stream, dst, src);
    return hipGetLastError();
}

hipError_t launch_zero(xsum_acc_t *acc, uint64_t count, hipStream_t stream)
{
    const uint64_t words = count * (sizeof(xsum_acc_t) / 8);
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       (uint64_t *)acc, words);
    return hipGetLastError();
}

}  // namespace xsum
