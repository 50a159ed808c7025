// Segmented exact sums: many independent sums, of uneven lengths and mixed
// formats, in one persistent launch (Section 6 of Goodrich & Eldawy: every
// reducer sums its own numbers into a superaccumulator; long inputs are first
// combined per chunk and the per-chunk states merged and rounded once).
//
// Work items come from a host-built plan, longest first, claimed by every
// wave from a shared queue (one device atomic per large item, one per few
// short items):
//   * lane group: up to 64 whole segments of one format and similar length
//     (the plan sorts segments by length).  Each lane streams its own segment
//     into its private LDS column exactly as the single-sum kernel does, then
//     carry-normalises and rounds it alone (finish_lane), so a segment costs
//     about 1/64 of a wave's fixed work.
//   * whole segment: a longer segment loaded coalesced by one wave, which
//     merges its 64 columns, carry-normalises and rounds with no state in
//     global memory and no device-scope fence.
//   * chunk: a contiguous run of a very long segment, loaded coalesced by a
//     wave.  The wave merges its 64 columns and adds the digits into the
//     segment's state with system-scope int64 atomics, which are performed
//     at the memory side past every XCD's L2; after they have completed it
//     takes a per-segment ticket, and the last chunk rounds the state (and
//     zeroes it for the next launch).  No cache write-back is needed, but
//     every chunk still pays a merge, its atomics and a ticket, so chunks
//     are large.
// The queue head and the exit counter return to zero at the end of every
// launch, so a launch can be replayed from a captured graph without memsets.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xsum.h"
#include "xsum_device.h"
#include "xsum_internal.h"
#include "xsum_segmented.h"

namespace xsum {


template <int FMT> struct LaneOut;
template <> struct LaneOut<XSUM_F64> { static constexpr int kNatural = XSUM_F64; };
template <> struct LaneOut<XSUM_F32> { static constexpr int kNatural = XSUM_F32; };
template <> struct LaneOut<XSUM_BF16> { static constexpr int kNatural = XSUM_F32; };

// Per-wave LDS: a 66-row column set (every format uses all of it) and a
// 68-digit merge vector.
struct WaveLds {
    uint64_t cols[Geo<XSUM_F64>::kN][64];
    int64_t merged[kDigits];
};

template <int FMT>
__device__ __forceinline__ void zero_column(uint64_t *col)
{
#pragma unroll
    for (int d = 0; d < Geo<FMT>::kN; ++d)
        lds_store(col + d * 64, 0);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        v = max(v, (uint32_t)__shfl_xor(v, s, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        v |= (uint32_t)__shfl_xor(v, s, 64);
    return v;
}

// Two-pass rounding of one lane's digits held in rows [r0, r1) of its
// column (row d at col[d * 64] is digit digit0 + d, weight
// 2^(32 (digit0 + d)) in units of 2^-1074); every other row of the column is
// zero.  Pass 1 carries the raw digits upward and writes the canonical
// digits back, noting the lowest non-zero digit z, the highest non-zero
// digit and the highest digit that is not all ones; the final carry is the
// sign.  r1 must leave room above the highest row that received chunks for
// the carries to settle (two rows).  Pass 2 reads the three digits the
// rounding needs: for a negative sum the magnitude's digits are 0 below z,
// 2^32 - u at z and 2^32 - 1 - u above it, so in both cases "any non-zero
// digit below h - 2" is simply z < h - 2.  Rows [r0, r1) are zeroed
// afterwards, so the whole column is zero again.
__device__ __forceinline__ uint64_t finish_lane_window(uint64_t *col, int r0, int r1,
                                                       int digit0, uint32_t special,
                                                       int out_fmt, uint32_t &flags)
{
    int64_t carry = 0;
    int z = -1, hnz = -1, hff = -1;
    for (int d = r0; d < r1; ++d) {
        const int64_t x = (int64_t)lds_load(col + d * 64) + carry;
        const uint32_t u = (uint32_t)((uint64_t)x & kLow32);
        carry = x >> 32;
        lds_store(col + d * 64, u);
        if (u != 0) {
            hnz = d;
            z = (z < 0) ? d : z;
        }
        if (u != 0xffffffffu)
            hff = d;
    }
    const OutFormat f = out_format(out_fmt);
    flags = 0;
    uint64_t bits;
    const bool negative = carry < 0;
    if (special_result(special, f, bits, flags)) {
    } else if (!(carry == 0 || carry == -1) || (negative && z < 0)) {
        // beyond the digits: far above every format's range
        flags = XSUM_FLAG_OVERFLOW | XSUM_FLAG_INEXACT;
        bits = fmt_inf(f, negative);
    } else if (!negative && hnz < 0) {
        bits = 0;                                   // exact zero -> +0
    } else {
        const int h = negative ? (hff > z ? hff : z) : hnz;
        uint32_t w[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int d = h - i;
            uint32_t u = d >= 0 ? (uint32_t)lds_load(col + (d >= 0 ? d : 0) * 64) : 0u;
            if (negative)
                u = d < z ? 0u : (d == z ? 0u - u : ~u);
            w[i] = u;
        }
        bits = round_magnitude(negative, digit0 + h, w[0], w[1], w[2], z < h - 2,
                               f, flags);
    }
    for (int d = r0; d < r1; ++d)
        lds_store(col + d * 64, 0);
    return bits;
}

// Rows a lane's elements have touched, from the smallest and largest key it
// met (Section 2: a sparse superaccumulator keeps only its active
// components; a lane here keeps the bounds of its active rows).  Keys:
// binary64 the exponent field e (rows of digits k and k + 1, k = (max(e,1) -
// 1) >> 5); binned formats the magnitude bits a (the two entries of bin b).
// kmin > kmax means no element.
template <int FMT>
__device__ __forceinline__ uint32_t key_row_lo(uint32_t k)
{
    if constexpr (FMT == XSUM_F64)
        return (max(k, 1u) - 1u) >> 5;
    else if constexpr (FMT == XSUM_F32)
        return 2 * ((max(k, 0x00800000u) + (4u << 23)) >> 26);
    else
        return 2 * ((max(k, 0x80u) + 0x200u) >> 10);
}

template <int FMT>
__device__ __forceinline__ uint32_t key_row_hi(uint32_t k)
{
    return key_row_lo<FMT>(k) + 1;
}

// Running key bounds over the valid vectors of a step (vector j is valid for
// j < nvalid; the others are the zero padding of lanes past their share).
template <int FMT, int U>
__device__ __forceinline__ void track_keys(const vec4u (&q)[U], uint64_t nvalid,
                                           uint32_t &kmin, uint32_t &kmax)
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const bool ok = (uint64_t)j < nvalid;
        if constexpr (FMT == XSUM_F64) {
            const uint32_t e0 = (q[j].y >> 20) & 0x7ffu, e1 = (q[j].w >> 20) & 0x7ffu;
            kmin = min(kmin, ok ? min(e0, e1) : 0xffffffffu);
            kmax = max(kmax, ok ? max(e0, e1) : 0u);
        } else if constexpr (FMT == XSUM_F32) {
            const uint32_t a0 = q[j].x & 0x7fffffffu, a1 = q[j].y & 0x7fffffffu,
                           a2 = q[j].z & 0x7fffffffu, a3 = q[j].w & 0x7fffffffu;
            kmin = min(kmin, ok ? min(min(a0, a1), min(a2, a3)) : 0xffffffffu);
            kmax = max(kmax, ok ? max(max(a0, a1), max(a2, a3)) : 0u);
        } else {
            const vec4u m = q[j] & 0x7fff7fffu;
            const uint32_t lo = min(min(m.x & 0xffffu, m.y & 0xffffu),
                                    min(m.z & 0xffffu, m.w & 0xffffu));
            const uint32_t hi = min(min(m.x >> 16, m.y >> 16), min(m.z >> 16, m.w >> 16));
            const uint32_t mx = max(max(max(m.x & 0xffffu, m.y & 0xffffu),
                                        max(m.z & 0xffffu, m.w & 0xffffu)),
                                    max(max(m.x >> 16, m.y >> 16), max(m.z >> 16, m.w >> 16)));
            kmin = min(kmin, ok ? min(lo, hi) : 0xffffffffu);
            kmax = max(kmax, ok ? mx : 0u);
        }
    }
}

// One element given as its bit pattern (read earlier with a scalar load):
// added like add_scalar adds one read in place.
template <int FMT>
__device__ __forceinline__ void add_element(uint64_t bits, uint64_t *col, uint32_t &spec)
{
    uint32_t emax = 0;
    if constexpr (FMT == XSUM_F64) {
        const uint32_t lo = (uint32_t)bits, hi = (uint32_t)(bits >> 32);
        add_f64(lo, hi, col, emax);
        fix_f64(lo, hi, col, spec);
    } else if constexpr (FMT == XSUM_F32) {
        add_f32((uint32_t)bits, col, emax);
        fix_f32((uint32_t)bits, col, spec);
    } else {
        u16x2 em = (u16x2)0;
        add_bf16_pair((uint32_t)bits, col, em);    // upper half +0, adds 0
        fix_bf16_pair((uint32_t)bits, col, spec);
    }
}

template <int FMT>
__device__ __forceinline__ uint64_t load_element(const uint8_t *p)
{
    if constexpr (FMT == XSUM_F64)
        return *(const uint64_t *)p;
    else if constexpr (FMT == XSUM_F32)
        return *(const uint32_t *)p;
    else
        return *(const uint16_t *)p;
}

// The key (exponent field or magnitude bits) of an element's bit pattern.
template <int FMT>
__device__ __forceinline__ uint32_t element_key(uint64_t bits)
{
    if constexpr (FMT == XSUM_F64)
        return (uint32_t)(bits >> 52) & 0x7ffu;
    else if constexpr (FMT == XSUM_F32)
        return (uint32_t)bits & 0x7fffffffu;
    else
        return (uint32_t)bits & 0x7fffu;
}

// The elements of a segment outside its 16-byte vectors: the unaligned head
// and the ragged tail, fewer than one vector's worth each.  They are loaded
// when the work item starts, so their loads are in flight while the vectors
// stream, and added from registers at the end.
template <int FMT>
struct EdgeElems {
    static constexpr int kMax = 16 / Geo<FMT>::kBytes - 1;   // 1, 3 or 7
    uint64_t h[kMax], t[kMax];
    uint32_t nh, nt;

    __device__ __forceinline__ void load(const uint8_t *p, uint64_t head, uint64_t nv,
                                         uint64_t tail)
    {
        nh = (uint32_t)head;
        nt = (uint32_t)tail;
        const uint8_t *tp = p + head * Geo<FMT>::kBytes + nv * 16;
#pragma unroll
        for (int i = 0; i < kMax; ++i) {
            h[i] = 0;
            t[i] = 0;
            if ((uint32_t)i < nh)
                h[i] = load_element<FMT>(p + i * Geo<FMT>::kBytes);
            if ((uint32_t)i < nt)
                t[i] = load_element<FMT>(tp + i * Geo<FMT>::kBytes);
        }
    }

    __device__ __forceinline__ void add(uint64_t *col, uint32_t &spec, uint32_t &kmin,
                                        uint32_t &kmax)
    {
#pragma unroll
        for (int i = 0; i < kMax; ++i) {
            if ((uint32_t)i < nh) {
                const uint32_t k = element_key<FMT>(h[i]);
                kmin = min(kmin, k);
                kmax = max(kmax, k);
                add_element<FMT>(h[i], col, spec);
            }
            if ((uint32_t)i < nt) {
                const uint32_t k = element_key<FMT>(t[i]);
                kmin = min(kmin, k);
                kmax = max(kmax, k);
                add_element<FMT>(t[i], col, spec);
            }
        }
    }
};

// Carry step over rows [r0, r1) of a binary64 column: every row but the last
// keeps its low 32 bits, its carry goes to the row above; the carries of row
// r1 - 1 go to row r1.  The value is unchanged.
__device__ __forceinline__ void normalise_rows(uint64_t *col, int r0, int r1)
{
    int64_t carry = 0;
    for (int d = r0; d < r1; ++d) {
        const int64_t x = (int64_t)lds_load(col + d * 64) + carry;
        lds_store(col + d * 64, (uint64_t)x & kLow32);
        carry = x >> 32;
    }
    lds_store(col + r1 * 64, lds_load(col + r1 * 64) + (uint64_t)carry);
}

// Round the lane's own column, whose rows outside [r0, r1) are zero, and
// zero it.  binary64 columns are digits 0..65.  A binned column holds 33 bins
// of weight 2^(8(b + kBin0)), each as a positive and a negative entry; each
// bin's signed value is moved to its radix-2^32 digit (kBin0 / 4 onwards),
// written back over the entries it came from (digit kBin0 / 4 + i lands in
// entry i, never past an entry still to be read), split into 32-bit halves
// so no shift overflows; two digits above the last take any carry.
template <int FMT>
__device__ __forceinline__ uint64_t finish_lane(uint64_t *col, int r0, int r1,
                                                uint32_t spec, int out_fmt,
                                                uint32_t &flags)
{
    if constexpr (FMT == XSUM_F64) {
        // two rows above the highest that received chunks let carries settle
        return finish_lane_window(col, r0, min(r1 + 2, Geo<XSUM_F64>::kN), 0, spec,
                                  out_fmt, flags);
    } else {
        constexpr int kBin0 = Geo<FMT>::kBin0;
        constexpr int kDigit0 = kBin0 >> 2;
        if (r0 >= r1)
            return finish_lane_window(col, 0, 0, kDigit0, spec, out_fmt, flags);
        const int b0 = r0 >> 1, b1 = (r1 - 1) >> 1;   // bins b0..b1
        const int g0 = (b0 + kBin0) >> 2;
        int64_t cur = 0, nxt = 0;                  // digits g and g + 1
        int g_prev = g0;
        for (int b = b0; b <= b1; ++b) {
            const int g = (b + kBin0) >> 2;
            const int sh = 8 * ((b + kBin0) & 3);
            const int64_t v = (int64_t)lds_load(col + (2 * b) * 64) -
                              (int64_t)lds_load(col + (2 * b + 1) * 64);
            if (g != g_prev) {
                lds_store(col + (g_prev - kDigit0) * 64, (uint64_t)cur);
                cur = nxt;
                nxt = 0;
                g_prev = g;
            }
            const uint64_t lo = ((uint64_t)v & kLow32) << sh;     // < 2^56
            const int64_t hi = (int64_t)((uint64_t)(v >> 32) << sh);
            cur += (int64_t)(lo & kLow32);
            nxt += (int64_t)(lo >> 32) + hi;
        }
        // the last two digits, then two empty digits for the carry
        const int e1 = g_prev - kDigit0;
        lds_store(col + e1 * 64, (uint64_t)cur);
        lds_store(col + (e1 + 1) * 64, (uint64_t)nxt);
        lds_store(col + (e1 + 2) * 64, 0);
        lds_store(col + (e1 + 3) * 64, 0);
        const uint64_t bits = finish_lane_window(col, g0 - kDigit0, e1 + 4, kDigit0, spec,
                                                 out_fmt, flags);
        // bin entries above the digits were left as they were
        for (int d = e1 + 4; d < r1; ++d)
            lds_store(col + d * 64, 0);
        return bits;
    }
}

// Add the rows [r0, r1) of the NL - 1 columns to the right of this lane's
// into its own.  Every read of a row is independent, so the reads of a row
// are issued together.
template <int NL>
__device__ __forceinline__ void fold_columns(uint64_t *col, int r0, int r1)
{
    for (int d = r0; d < r1; ++d) {
        int64_t v = (int64_t)lds_load(col + d * 64);
#pragma unroll
        for (int k = 1; k < NL; ++k) {
            v += (int64_t)lds_load(col + d * 64 + k);
            lds_store(col + d * 64 + k, 0);
        }
        lds_store(col + d * 64, (uint64_t)v);
    }
}

// A lane's share of its segment in a lane group of 2^glog lanes per
// segment: every 2^glog-th 16-byte vector, starting at vector sub.
struct LaneShare {
    const uint8_t *p;       // the segment's first element
    const vec4u *vp;        // this lane's first vector
    uint64_t head, nv, tail, my_nv;
    uint32_t sub;
    bool live;
};

// ebytes_log2: log2 of the element size (3, 2 or 1).
__device__ __forceinline__ LaneShare lane_share(const uint8_t *base, const SegLane &e,
                                                uint32_t count, uint32_t glog,
                                                uint32_t ebytes_log2, int lane)
{
    LaneShare s;
    s.sub = (uint32_t)lane & ((1u << glog) - 1);
    s.live = ((uint32_t)lane >> glog) < count;
    const uint64_t off = s.live ? e.byte_offset : 0;
    const uint64_t L = s.live ? e.length : 0;
    s.p = base + off;
    s.head = (((16 - ((uintptr_t)s.p & 15)) & 15) >> ebytes_log2);
    if (s.head > L)
        s.head = L;
    s.nv = (L - s.head) >> (4 - ebytes_log2);
    s.tail = L - s.head - (s.nv << (4 - ebytes_log2));
    s.vp = (const vec4u *)(s.p + (s.head << ebytes_log2)) + s.sub;
    s.my_nv = s.nv > s.sub ? ((s.nv - s.sub - 1) >> glog) + 1 : 0;
    return s;
}

// Step `it` of a lane's share: its vectors it*UL .. it*UL + UL - 1 (zero
// vectors past the end).  Every lane loads on every step (no load sits in a
// branch, so the compiler's wait counts keep a spare buffer's loads in
// flight).  In a step where every lane's share is either whole or over, a
// lane's loads walk one pointer by a fixed stride (zero for a lane that
// reads the zero vector); only a step that ends some lane's share inside it
// picks an address per vector.
__device__ __forceinline__ bool whole_step(uint64_t my_nv, uint32_t it, int ul)
{
    const int64_t rem = (int64_t)my_nv - (int64_t)it * ul;
    return __ballot(rem > 0 && rem < ul) == 0;
}

template <int UL, int CAP>
__device__ __forceinline__ void load_lane_step(vec4u (&q)[CAP], const vec4u *vp,
                                               uint64_t my_nv, uint32_t it, uint32_t glog,
                                               const vec4u *zero)
{
    static_assert(UL <= CAP, "buffer too small");
    const int64_t rem = (int64_t)my_nv - (int64_t)it * UL;
    if (whole_step(my_nv, it, UL)) {
        const uint8_t *a = rem > 0 ? (const uint8_t *)(vp + ((uint64_t)it * UL << glog))
                                   : (const uint8_t *)zero;
        const uint64_t st = rem > 0 ? (16ull << glog) : 0;
#pragma unroll
        for (int j = 0; j < UL; ++j) {
            q[j] = *(const vec4u *)a;   // cached: neighbouring loads share lines
            a += st;
        }
    } else {
#pragma unroll
        for (int j = 0; j < UL; ++j) {
            const uint64_t i = (uint64_t)it * UL + j;
            const vec4u *src = i < my_nv ? vp + (i << glog) : zero;
            q[j] = *src;
        }
    }
}

// One lane group: 2^glog lanes share each segment (64 >> glog segments, the
// first `count` valid).  Lane l reads every 2^glog-th 16-byte vector of
// segment l >> glog, starting at vector l mod 2^glog, into its own column, so
// a load instruction touches 64 >> glog runs of 2^glog contiguous vectors
// instead of 64 scattered ones.  Each lane keeps the bounds of the rows its
// elements touched, and every later step (carry steps, the fold of a
// segment's columns into its first lane's, the rounding and the clearing)
// works on those rows only: short segments of data with a narrow exponent
// range touch a few of the 66 rows.
template <int FMT, int UL>
__device__ __forceinline__ void run_lane_group(const uint8_t *base, const SegLane &e,
                                               uint32_t count, uint32_t glog,
                                               uint64_t *col, int out_mode,
                                               uint64_t *out, uint32_t *flags,
                                               const vec4u *zero, int lane)
{
    using G = Geo<FMT>;
    constexpr uint32_t kLog2Bytes = FMT == XSUM_F64 ? 3 : FMT == XSUM_F32 ? 2 : 1;
    const LaneShare sh = lane_share(base, e, count, glog, kLog2Bytes, lane);
    const uint32_t sub = sh.sub;
    const bool live = sh.live;
    const uint32_t s = e.seg;
    const uint8_t *p = sh.p;
    const uint64_t head = sh.head, nv = sh.nv, tail = sh.tail;
    const vec4u *vp = sh.vp;
    const uint64_t my_nv = sh.my_nv;
    uint32_t spec = 0;
    uint32_t kmin = 0xffffffffu, kmax = 0;
    EdgeElems<FMT> edges;
    edges.load(p, sub == 0 ? head : 0, nv, sub == 0 ? tail : 0);

    const uint64_t my_iters = (my_nv + UL - 1) / UL;
    const uint32_t iters = wave_max_u32((uint32_t)my_iters);
    // binary64: at most 1024 + 2*UL + 2 elements between carry steps
    constexpr int kNormIters = 512 / UL;
    int since = 0;
    // each lane walks its share of its segment, UL vectors per step, the next
    // step's loads in flight while the current step is added
    vec4u qa[UL], qb[UL];
    auto step_rem = [&](uint32_t it) -> int64_t {
        return (int64_t)my_nv - (int64_t)it * UL;
    };
    auto uniform_step = [&](int64_t rem) -> bool {
        return __ballot(rem > 0 && rem < UL) == 0;
    };
    auto load_step = [&](vec4u (&q)[UL], uint32_t it) {
        load_lane_step<UL>(q, vp, my_nv, it, glog, zero);
    };
    auto add_step = [&](const vec4u (&q)[UL], uint32_t it) {
        const int64_t rem = step_rem(it);
        if (uniform_step(rem)) {
            // whole step or none: bounds of all UL vectors, kept or dropped
            uint32_t smin = 0xffffffffu, smax = 0;
            track_keys<FMT, UL>(q, UL, smin, smax);
            kmin = min(kmin, rem > 0 ? smin : 0xffffffffu);
            kmax = max(kmax, rem > 0 ? smax : 0u);
        } else {
            track_keys<FMT, UL>(q, rem > 0 ? (uint64_t)rem : 0, kmin, kmax);
        }
        add_tile<FMT, UL>(q, col, spec);
        if constexpr (FMT == XSUM_F64) {
            if (++since >= kNormIters) {
                // rows below the lowest and above the highest touched one
                // (plus the carry row) are zero
                normalise_rows(col, (int)key_row_lo<FMT>(kmin),
                               min((int)key_row_hi<FMT>(kmax) + 1, G::kN - 1));
                since = 0;
            }
        }
    };
    // as in accumulate_span, the spare buffer is loaded on every pass (past
    // the last step, with zeros, never added)
    if (iters > 0)
        load_step(qa, 0);
    for (uint32_t it = 0; it < iters; it += 2) {
        load_step(qb, it + 1);
        add_step(qa, it);
        if (it + 1 >= iters)
            break;
        load_step(qa, it + 2);
        add_step(qb, it + 1);
    }
    edges.add(col, spec, kmin, kmax);
    // the rows this lane may have written: binary64 also the carry row above
    // the highest touched one
    int r0 = G::kN, r1 = 0;
    if (kmin <= kmax) {
        r0 = (int)key_row_lo<FMT>(kmin);
        r1 = (int)key_row_hi<FMT>(kmax) + 1;
        if constexpr (FMT == XSUM_F64)
            r1 = min(r1 + 1, G::kN);
    }
    if (glog > 0) {
        // the segment's lanes are neighbours: fold their columns into the
        // first one.  Binary64 columns get a carry step first (entries below
        // 2^32, the row above holding only carries), so a sum of up to 16
        // entries cannot overflow; binary32 bins hold at most lane_max
        // chunks below 2^31 each.
        for (uint32_t k = 1; k < (1u << glog); k <<= 1)
            spec |= (uint32_t)__shfl_xor((int)spec, (int)k, 64);
        if constexpr (FMT == XSUM_F64) {
            if (r0 < r1) {
                const int top = min(r1, G::kN - 1);
                normalise_rows(col, r0, top);
                r1 = top + 1;
            }
        }
        for (uint32_t k = 1; k < (1u << glog); k <<= 1) {
            r0 = min(r0, __shfl_xor(r0, (int)k, 64));
            r1 = max(r1, __shfl_xor(r1, (int)k, 64));
        }
        wave_lds_fence();
        if (sub == 0) {
            if (glog == 1)
                fold_columns<2>(col, r0, r1);
            else if (glog == 2)
                fold_columns<4>(col, r0, r1);
            else if (glog == 3)
                fold_columns<8>(col, r0, r1);
            else
                fold_columns<16>(col, r0, r1);
        }
        wave_lds_fence();
        if (sub != 0) {         // folded into the first lane and cleared
            r0 = G::kN;
            r1 = 0;
        }
    }

    const int of = out_mode == XSUM_SAME ? LaneOut<FMT>::kNatural : out_mode;
    uint32_t fl;
    // every lane rounds (and clears) its own rows; only a segment's first
    // lane holds the whole sum and writes it
    const uint64_t bits = finish_lane<FMT>(col, r0, r1, spec, of, fl);
    if (live && sub == 0) {
        out[s] = bits;
        if (flags)
            flags[s] = fl;
    }
}

// Add nv 16-byte vectors starting at vp (wave-contiguous tiles of 64*UC
// vectors, the next tile in flight), plus the segment's head and tail
// elements when asked, into the lanes' columns.
template <int FMT, int UC>
__device__ __forceinline__ void accumulate_span(const vec4u *vp, uint64_t nv,
                                                const uint8_t *head_p,
                                                uint64_t head,
                                                const uint8_t *tail_p,
                                                uint64_t tail, uint64_t *col,
                                                uint32_t &spec, int lane)
{
    using G = Geo<FMT>;
    constexpr uint64_t kTile = 64ull * UC;
    constexpr int kNormTiles = 512 / UC;
    const uint64_t full = nv / kTile;
    int since = 0;
    // one head and one tail element per lane, loaded now, added at the end
    uint64_t hv = 0, tv = 0;
    if ((uint64_t)lane < head)
        hv = load_element<FMT>(head_p + (uint64_t)lane * G::kBytes);
    if ((uint64_t)lane < tail)
        tv = load_element<FMT>(tail_p + (uint64_t)lane * G::kBytes);
    if (full > 0) {
        // The next tile's loads are issued on every pass: past the span's
        // last full tile every one of them re-reads the lane's vector of the
        // tile just loaded (a cache hit) into the spare buffer, which is
        // never added.  With no load skipped, the compiler's wait counts
        // leave the spare buffer's loads in flight while the current tile is
        // added; a skipped load would force a wait for every load issued.
        vec4u qa[UC], qb[UC];
#pragma unroll
        for (int j = 0; j < UC; ++j)
            qa[j] = __builtin_nontemporal_load(vp + j * 64 + lane);
        for (uint64_t tt = 0; tt < full; tt += 2) {
            const bool more_b = tt + 1 < full;
            const vec4u *pb = vp + (more_b ? tt + 1 : tt) * kTile + lane;
            const uint64_t sb = more_b ? 64 : 0;
#pragma unroll
            for (int j = 0; j < UC; ++j)
                qb[j] = __builtin_nontemporal_load(pb + j * sb);
            add_tile<FMT, UC>(qa, col, spec);
            if (!more_b)
                break;
            const bool more_a = tt + 2 < full;
            const vec4u *pa = vp + (more_a ? tt + 2 : tt + 1) * kTile + lane;
            const uint64_t sa = more_a ? 64 : 0;
#pragma unroll
            for (int j = 0; j < UC; ++j)
                qa[j] = __builtin_nontemporal_load(pa + j * sa);
            add_tile<FMT, UC>(qb, col, spec);
            if constexpr (FMT == XSUM_F64) {
                since += 2;
                if (since >= kNormTiles) {
                    normalise_column<G::kN>(col);
                    since = 0;
                }
            }
        }
    }
    // the last partial tile: all its loads issued before any is consumed
    {
        vec4u q[UC];
#pragma unroll
        for (int j = 0; j < UC; ++j) {
            const uint64_t i = full * kTile + (uint64_t)j * 64 + lane;
            q[j] = vec4u{0u, 0u, 0u, 0u};
            if (i < nv)
                q[j] = __builtin_nontemporal_load(vp + i);
        }
        add_tile<FMT, UC>(q, col, spec);
    }
    if ((uint64_t)lane < head)
        add_element<FMT>(hv, col, spec);
    if ((uint64_t)lane < tail)
        add_element<FMT>(tv, col, spec);
}

// Merge the wave's 64 columns into w.merged, then clear the columns.
template <int FMT>
__device__ __forceinline__ void merge_and_clear(WaveLds &w, uint64_t *col,
                                                int lane)
{
    for (int d = lane; d < kDigits; d += 64)
        w.merged[d] = 0;
    wave_lds_fence();
    merge_wave_columns<FMT>(w.cols, w.merged, lane);
    wave_lds_fence();
    zero_column<FMT>(col);
}

struct SpanGeom {
    const uint8_t *p;
    uint64_t head, nvs, tail;
};

template <int FMT>
__device__ __forceinline__ SpanGeom span_geom(const uint8_t *base,
                                              const SegDesc &d)
{
    using G = Geo<FMT>;
    SpanGeom g;
    g.p = base + d.byte_offset;
    const uint64_t L = d.length;
    g.head = ((16 - ((uintptr_t)g.p & 15)) & 15) / G::kBytes;
    if (g.head > L)
        g.head = L;
    g.nvs = (L - g.head) / G::kPerVec;
    g.tail = L - g.head - g.nvs * G::kPerVec;
    return g;
}

// One whole segment, summed, normalised and rounded by one wave.  Its offset
// and length travel in the work item itself.
template <int FMT, int UC>
__device__ __forceinline__ void run_whole(const uint8_t *base, const SegTask &t,
                                          WaveLds &w, uint64_t *col, int out_mode,
                                          uint64_t *out, uint32_t *flags, int lane)
{
    using G = Geo<FMT>;
    const uint32_t s = t.a;
    const SegDesc d{t.v0, t.nv, 0, 0};
    const SpanGeom g = span_geom<FMT>(base, d);
    const vec4u *vp = (const vec4u *)(g.p + g.head * G::kBytes);
    uint32_t spec = 0;
    accumulate_span<FMT, UC>(vp, g.nvs, g.p, g.head,
                             g.p + g.head * G::kBytes + g.nvs * 16, g.tail, col,
                             spec, lane);
    merge_and_clear<FMT>(w, col, lane);
    spec = wave_or_u32(spec);
    int64_t a = 0, b = 0;
    if (lane <= 33) {
        a = w.merged[2 * lane];
        b = w.merged[2 * lane + 1];
    }
    normalise_wave(a, b, lane);
    const int of = out_mode == XSUM_SAME ? LaneOut<FMT>::kNatural : out_mode;
    uint32_t fl;
    const uint64_t bits = round_wave(a, b, lane, spec, of, fl);
    if (lane == 0) {
        out[s] = bits;
        if (flags)
            flags[s] = fl;
    }
}

// One chunk of a very long segment, summed by the whole wave.
template <int FMT, int UC>
__device__ __forceinline__ void run_chunk(const uint8_t *base, const SegDesc *segs,
                          const SegTask &t, xsum_acc_t *states, WaveLds &w,
                          uint64_t *col, int out_mode, uint64_t *out,
                          uint32_t *flags, int lane)
{
    using G = Geo<FMT>;
    const uint32_t s = t.a;
    const uint32_t cflags = t.kind_dtype_flags >> 16;
    const SpanGeom g = span_geom<FMT>(base, segs[s]);
    const vec4u *vp = (const vec4u *)(g.p + g.head * G::kBytes) + t.v0;
    uint32_t spec = 0;
    accumulate_span<FMT, UC>(vp, t.nv, g.p, (cflags & kChunkFirst) ? g.head : 0,
                             g.p + g.head * G::kBytes + g.nvs * 16,
                             (cflags & kChunkLast) ? g.tail : 0, col, spec, lane);
    merge_and_clear<FMT>(w, col, lane);
    spec = wave_or_u32(spec);

    // The chunk's digits go to the segment's state with system-scope atomics
    // (performed past the L2s, so no write-back fence is needed); the wave
    // waits until they have completed before it takes its ticket, and the
    // wave with the last ticket reads the state with system-scope atomics.
    xsum_acc_t *st = &states[t.b];
    for (int d = lane; d < kDigits; d += 64) {
        const int64_t dv = w.merged[d];
        if (dv)
            __hip_atomic_fetch_add(&st->digit[d], dv, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (lane == 0 && spec)
        __hip_atomic_fetch_or(&st->special, spec, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    uint32_t ticket = 0;
    if (lane == 0)
        ticket = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_SYSTEM);
    ticket = __shfl(ticket, 0, 64);
    if (ticket == t.nchunks - 1) {
        const int of = out_mode == XSUM_SAME ? LaneOut<FMT>::kNatural : out_mode;
        Finish fin{kRound, of, out + s, flags ? flags + s : nullptr, 1};
        finish_state<true>(st, fin, lane);
    }
}

// The lane entry of work item t for this lane: that of its segment, lane
// >> glog (zero when t is not a lane group or the segment is past its count).
__device__ __forceinline__ SegLane lane_entry(const SegLane *__restrict__ lanes,
                                              const SegTask &t, uint32_t ntasks_left,
                                              int lane)
{
    SegLane e{0, 0, 0};
    const uint32_t seg = (uint32_t)lane >> ((t.kind_dtype_flags >> 16) & kLaneGlogMask);
    if (ntasks_left && (t.kind_dtype_flags & 0xffu) == kLaneGroup && seg < t.b)
        e = lanes[t.a + seg];
    return e;
}

template <int WAVES, int UL, int UC>
__global__ __launch_bounds__(WAVES * 64) void segmented_kernel(
    const uint8_t *__restrict__ base, const SegDesc *__restrict__ segs,
    const SegTask *__restrict__ tasks, uint32_t ntasks,
    const SegLane *__restrict__ lanes, xsum_acc_t *states, SegCtl *ctl,
    int out_mode, uint64_t *out, uint32_t *flags)
{
    __shared__ WaveLds lds[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds &w = lds[wave];
    uint64_t *col = &w.cols[0][lane];
    zero_column<XSUM_F64>(col);

    // Items are claimed from the queue one at a time, one item ahead: the
    // claim of the item after next is issued when an item starts, so its
    // round trip (a device-scope atomic takes microseconds) is hidden behind
    // a whole item, and a wave never holds more than the item it runs and
    // the one it has claimed.  Holding more (deeper prefetch, claims of
    // several short items at once) left waves idle at the end of the queue
    // while others still worked through items they had reserved.
    auto claim = [&]() -> uint32_t {
        uint32_t c = 0;
        if (lane == 0)
            c = atomicAdd(&ctl->head, 1u);
        return __shfl(c, 0, 64);
    };
    uint32_t cur = claim();
    uint32_t next = claim();
    SegTask t{};
    if (cur < ntasks)
        t = tasks[cur];
    SegLane e = lane_entry(lanes, t, cur < ntasks, lane);
    while (cur < ntasks) {
        const uint32_t kind = t.kind_dtype_flags & 0xffu;
        const uint32_t dtype = (t.kind_dtype_flags >> 8) & 0xffu;
        if (kind == kLaneGroup) {
            const uint32_t glog = (t.kind_dtype_flags >> 16) & kLaneGlogMask;
            const vec4u *zero = (const vec4u *)ctl->zero;
            if ((t.kind_dtype_flags >> 16) & kLaneUnroll8) {
                if (dtype == XSUM_F64)
                    run_lane_group<XSUM_F64, UL / 2>(base, e, t.b, glog, col, out_mode, out,
                                                      flags, zero, lane);
                else if (dtype == XSUM_F32)
                    run_lane_group<XSUM_F32, UL / 2>(base, e, t.b, glog, col, out_mode, out,
                                                      flags, zero, lane);
                else
                    run_lane_group<XSUM_BF16, UL / 2>(base, e, t.b, glog, col, out_mode, out,
                                                       flags, zero, lane);
            } else {
                if (dtype == XSUM_F64)
                    run_lane_group<XSUM_F64, UL>(base, e, t.b, glog, col, out_mode, out, flags,
                                                  zero, lane);
                else if (dtype == XSUM_F32)
                    run_lane_group<XSUM_F32, UL>(base, e, t.b, glog, col, out_mode, out, flags,
                                                  zero, lane);
                else
                    run_lane_group<XSUM_BF16, UL>(base, e, t.b, glog, col, out_mode, out, flags,
                                                   zero, lane);
            }
        } else if (kind == kWhole) {
            if (dtype == XSUM_F64)
                run_whole<XSUM_F64, UC>(base, t, w, col, out_mode, out, flags, lane);
            else if (dtype == XSUM_F32)
                run_whole<XSUM_F32, UC>(base, t, w, col, out_mode, out, flags, lane);
            else
                run_whole<XSUM_BF16, UC>(base, t, w, col, out_mode, out, flags, lane);
        } else {
            if (dtype == XSUM_F64)
                run_chunk<XSUM_F64, UC>(base, segs, t, states, w, col, out_mode, out, flags, lane);
            else if (dtype == XSUM_F32)
                run_chunk<XSUM_F32, UC>(base, segs, t, states, w, col, out_mode, out, flags, lane);
            else
                run_chunk<XSUM_BF16, UC>(base, segs, t, states, w, col, out_mode, out, flags, lane);
        }
        // the next item's record and lane entry, then the claim after it
        SegTask nt{};
        if (next < ntasks)
            nt = tasks[next];
        const SegLane ne = lane_entry(lanes, nt, next < ntasks, lane);
        const uint32_t following = claim();
        cur = next;
        next = following;
        t = nt;
        e = ne;
    }
    // The last wave out resets the queue for the next launch.  Every wave's
    // claims have returned before its exit increment is issued (each result
    // was read above), so no fence is needed here.
    if (lane == 0) {
        const uint32_t total = gridDim.x * WAVES;
        if (atomicAdd(&ctl->done, 1u) == total - 1) {
            __hip_atomic_store(&ctl->head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------ serving batches --
//
// One launch adds every chunk of every item of a batch into the item's
// destination state (Section 6: reducers accumulate into superaccumulators
// that are merged later; here the state persists across launches and is
// rounded by batch_finalize_kernel once the request is complete).  Task t is
// chunk t - first_task of the item found by binary search over first_task.

template <int FMT, int UC>
__device__ __forceinline__ void run_batch_chunk(const BatchItem &it, uint64_t c,
                                                uint64_t chunk_vectors,
                                                xsum_acc_t *states, WaveLds &w,
                                                uint64_t *col, int lane)
{
    using G = Geo<FMT>;
    const SegDesc d{0, it.length, it.dtype, 0};
    const SpanGeom g = span_geom<FMT>((const uint8_t *)it.ptr, d);
    const uint64_t v0 = c * chunk_vectors;
    const uint64_t nv = v0 < g.nvs ? min(chunk_vectors, g.nvs - v0) : 0;
    const uint64_t nch = g.nvs == 0 ? 1 : (g.nvs + chunk_vectors - 1) / chunk_vectors;
    const vec4u *vp = (const vec4u *)(g.p + g.head * G::kBytes) + v0;
    uint32_t spec = 0;
    accumulate_span<FMT, UC>(vp, nv, g.p, c == 0 ? g.head : 0,
                             g.p + g.head * G::kBytes + g.nvs * 16,
                             c + 1 == nch ? g.tail : 0, col, spec, lane);
    merge_and_clear<FMT>(w, col, lane);
    spec = wave_or_u32(spec);
    xsum_acc_t *st = &states[it.slot];
    for (int k = lane; k < kDigits; k += 64) {
        const int64_t dv = w.merged[k];
        if (dv)
            atomicAdd((unsigned long long *)&st->digit[k], (unsigned long long)dv);
    }
    if (lane == 0 && spec)
        atomicOr(&st->special, spec);
}

template <int UC>
__global__ __launch_bounds__(64) void batch_add_kernel(
    const BatchItem *__restrict__ items, uint32_t nitems, uint64_t ntasks,
    uint64_t chunk_vectors, xsum_acc_t *states, SegCtl *ctl)
{
    __shared__ WaveLds w;
    const int lane = threadIdx.x;
    uint64_t *col = &w.cols[0][lane];
    zero_column<XSUM_F64>(col);
    for (;;) {
        uint32_t t32 = 0;
        if (lane == 0)
            t32 = atomicAdd(&ctl->head, 1u);
        const uint64_t t = __shfl(t32, 0, 64);
        if (t >= ntasks)
            break;
        // last item whose first_task <= t
        uint32_t lo = 0, hi = nitems;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (items[mid].first_task <= t)
                lo = mid;
            else
                hi = mid;
        }
        const BatchItem it = items[lo];
        const uint64_t c = t - it.first_task;
        if (it.dtype == XSUM_F64)
            run_batch_chunk<XSUM_F64, UC>(it, c, chunk_vectors, states, w, col, lane);
        else if (it.dtype == XSUM_F32)
            run_batch_chunk<XSUM_F32, UC>(it, c, chunk_vectors, states, w, col, lane);
        else
            run_batch_chunk<XSUM_BF16, UC>(it, c, chunk_vectors, states, w, col, lane);
    }
    if (lane == 0) {
        const uint32_t total = gridDim.x;
        if (atomicAdd(&ctl->done, 1u) == total - 1) {
            __hip_atomic_store(&ctl->head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// One wave per entry: round states[slots[i]] to its format, write out[i] /
// flags[i] (8-byte slots), then zero the state for the next request.
__global__ __launch_bounds__(64) void batch_finalize_kernel(
    const uint32_t *__restrict__ slots, const uint32_t *__restrict__ fmts,
    uint32_t n, xsum_acc_t *states, uint64_t *out, uint32_t *flags)
{
    const uint32_t i = blockIdx.x;
    if (i >= n)
        return;
    const int lane = threadIdx.x;
    xsum_acc_t *st = &states[slots[i]];
    Finish fin{kRound, (int)fmts[i], out + i, flags ? flags + i : nullptr, 1};
    finish_state<false>(st, fin, lane);
}

hipError_t launch_batch_add(const BatchItem *items, uint32_t nitems,
                            uint64_t ntasks, uint64_t chunk_vectors,
                            xsum_acc_t *states, SegCtl *ctl, int blocks,
                            hipStream_t stream)
{
    hipLaunchKernelGGL((batch_add_kernel<16>), dim3((unsigned)blocks), dim3(64), 0,
                       stream, items, nitems, ntasks, chunk_vectors, states, ctl);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const uint32_t *slots, const uint32_t *fmts,
                                 uint32_t n, xsum_acc_t *states, uint64_t *out,
                                 uint32_t *flags, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(n), dim3(64), 0, stream, slots,
                       fmts, n, states, out, flags);
    return hipGetLastError();
}

static constexpr int kSegWaves = 1;
static constexpr int kSegLaneUnroll = 16;
static constexpr int kSegChunkUnroll = 16;
static constexpr int kSegBlocksPerCu = 4;

int segmented_blocks(int cu_count, int blocks_per_cu)
{
    return (blocks_per_cu > 0 ? blocks_per_cu : kSegBlocksPerCu) * cu_count;
}

hipError_t launch_segmented(const void *base, const SegDesc *segs,
                            const SegTask *tasks, uint32_t ntasks,
                            const SegLane *lanes, xsum_acc_t *states,
                            SegCtl *ctl, int out_mode, uint64_t *out,
                            uint32_t *flags, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((segmented_kernel<kSegWaves, kSegLaneUnroll, kSegChunkUnroll>),
                       dim3((unsigned)blocks), dim3(kSegWaves * 64), 0, stream,
                       (const uint8_t *)base, segs, tasks, ntasks, lanes, states,
                       ctl, out_mode, out, flags);
    return hipGetLastError();
}

uint64_t segmented_chunk_vectors() { return 1ull << 16; }  // 1 MiB

}  // namespace xsum
