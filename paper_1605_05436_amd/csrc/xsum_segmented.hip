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

// Work items claimed per queue atomic by the segmented kernel.
static constexpr int kSegPopBatch = 4;

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

// Round the lane's own column and zero it.  binary64 columns are digits
// 0..65.  A binned column holds 33 bins of weight 2^(8(b + kBin0)), each as a
// positive and a negative entry; each bin's signed value is moved to its
// radix-2^32 digit (kBin0 / 4 onwards), written back over the entries it came
// from (digit kBin0 / 4 + i lands in entry i, never past an entry still to be
// read), split into 32-bit halves so no shift overflows; two top digits take
// any carry.
template <int FMT>
__device__ __forceinline__ uint64_t finish_lane(uint64_t *col, uint32_t spec,
                                                int out_fmt, uint32_t &flags)
{
    if constexpr (FMT == XSUM_F64) {
        return finish_lane_digits<Geo<XSUM_F64>::kN>(col, 0, spec, out_fmt, flags);
    } else {
        constexpr int kBin0 = Geo<FMT>::kBin0;
        constexpr int kDigit0 = kBin0 >> 2;
        int64_t cur = 0, nxt = 0;                  // digits g and g + 1
        int g_prev = kDigit0;
#pragma unroll
        for (int b = 0; b < Geo<FMT>::kBins; ++b) {
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
        constexpr int kLast = (Geo<FMT>::kBins - 1 + kBin0) >> 2;
        lds_store(col + (kLast - kDigit0) * 64, (uint64_t)cur);
        lds_store(col + (kLast + 1 - kDigit0) * 64, (uint64_t)nxt);
        lds_store(col + (kLast + 2 - kDigit0) * 64, 0);
        lds_store(col + (kLast + 3 - kDigit0) * 64, 0);
        const uint64_t bits = finish_lane_digits<kLast + 4 - kDigit0>(col, kDigit0, spec,
                                                                      out_fmt, flags);
        // entries above the digits were left as they were
#pragma unroll
        for (int b = kLast + 4 - kDigit0; b < Geo<FMT>::kN; ++b)
            lds_store(col + b * 64, 0);
        return bits;
    }
}

// Add the entries of the NL - 1 columns to the right of this lane's into its
// own.  Every read is independent, so the rows are unrolled and the reads
// issued in batches.
template <int N, int NL>
__device__ __forceinline__ void fold_columns(uint64_t *col)
{
#pragma unroll
    for (int d = 0; d < N; ++d) {
        int64_t v = (int64_t)lds_load(col + d * 64);
#pragma unroll
        for (int k = 1; k < NL; ++k)
            v += (int64_t)lds_load(col + d * 64 + k);
        lds_store(col + d * 64, (uint64_t)v);
    }
}

// One lane group: 2^glog lanes share each segment (64 >> glog segments, the
// first `count` valid).  Lane l reads every 2^glog-th 16-byte vector of
// segment l >> glog, starting at vector l mod 2^glog, into its own column, so
// a load instruction touches 64 >> glog runs of 2^glog contiguous vectors
// instead of 64 scattered ones.  The columns of a segment's lanes are then
// carry-normalised, summed into its first lane's column, and rounded there.
template <int FMT, int UL>
__device__ __forceinline__ void run_lane_group(const uint8_t *base, const SegLane &e,
                                               uint32_t count, uint32_t glog,
                                               uint64_t *col, int out_mode,
                                               uint64_t *out, uint32_t *flags,
                                               const vec4u *zero, int lane)
{
    using G = Geo<FMT>;
    const uint32_t sub = (uint32_t)lane & ((1u << glog) - 1);
    const bool live = ((uint32_t)lane >> glog) < count;
    const uint32_t s = e.seg;
    const uint64_t off = live ? e.byte_offset : 0;
    const uint64_t L = live ? e.length : 0;
    const uint8_t *p = base + off;
    uint64_t head = ((16 - ((uintptr_t)p & 15)) & 15) / G::kBytes;
    if (head > L)
        head = L;
    const uint64_t nv = (L - head) / G::kPerVec;
    const uint64_t tail = L - head - nv * G::kPerVec;
    const vec4u *vp = (const vec4u *)(p + head * G::kBytes) + sub;
    // this lane's vectors: sub, sub + 2^glog, ...
    const uint64_t my_nv = nv > sub ? ((nv - sub - 1) >> glog) + 1 : 0;
    uint32_t spec = 0;

    const uint64_t my_iters = (my_nv + UL - 1) / UL;
    const uint32_t iters = wave_max_u32((uint32_t)my_iters);
    // binary64: at most 1024 + 2*UL + 2 elements between normalisations
    constexpr int kNormIters = 512 / UL;
    int since = 0;
    // each lane walks its share of its segment, UL vectors per step, the next
    // step's loads in flight while the current step is added
    vec4u qa[UL], qb[UL];
    // Every lane loads on every step (no load sits in a branch, so the
    // compiler's wait counts keep the spare buffer's loads in flight): a
    // lane past the end of its share, or a step past the last, loads the
    // zero vector instead.
    auto load_step = [&](vec4u (&q)[UL], uint32_t it) {
#pragma unroll
        for (int j = 0; j < UL; ++j) {
            const uint64_t i = (uint64_t)it * UL + j;
            const vec4u *src = i < my_nv ? vp + (i << glog) : zero;
            q[j] = *src;    // cached: neighbouring loads share lines
        }
    };
    auto norm_step = [&]() {
        if constexpr (FMT == XSUM_F64) {
            if (++since >= kNormIters) {
                normalise_column<G::kN>(col);
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
        add_tile<FMT, UL>(qa, col, spec);
        norm_step();
        if (it + 1 >= iters)
            break;
        load_step(qa, it + 2);
        add_tile<FMT, UL>(qb, col, spec);
        norm_step();
    }
    if (sub == 0) {
        for (uint64_t i = 0; i < head; ++i)
            add_scalar<FMT>(p + i * G::kBytes, col, spec);
        const uint8_t *tp = p + head * G::kBytes + nv * 16;
        for (uint64_t i = 0; i < tail; ++i)
            add_scalar<FMT>(tp + i * G::kBytes, col, spec);
    }
    if (glog > 0) {
        // the segment's lanes are neighbours: fold their columns into the
        // first one.  Binary64 columns are carry-normalised first (entries
        // below 2^32, the last one holding only carries), so a sum of up to
        // four entries cannot overflow; binary32 bins hold at most lane_max
        // chunks below 2^31 each.
        for (uint32_t k = 1; k < (1u << glog); k <<= 1)
            spec |= (uint32_t)__shfl_xor((int)spec, (int)k, 64);
        if constexpr (FMT == XSUM_F64)
            normalise_column<G::kN>(col);
        wave_lds_fence();
        if (sub == 0) {
            if (glog == 1)
                fold_columns<G::kN, 2>(col);
            else
                fold_columns<G::kN, 4>(col);
        }
        wave_lds_fence();
    }

    const int of = out_mode == XSUM_SAME ? LaneOut<FMT>::kNatural : out_mode;
    uint32_t fl;
    // every lane rounds (and clears) its own column; only a segment's first
    // lane holds the whole sum and writes it
    const uint64_t bits = finish_lane<FMT>(col, spec, of, fl);
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
        add_scalar<FMT>(head_p + (uint64_t)lane * G::kBytes, col, spec);
    if ((uint64_t)lane < tail)
        add_scalar<FMT>(tail_p + (uint64_t)lane * G::kBytes, col, spec);
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
    const uint32_t seg = (uint32_t)lane >> (t.kind_dtype_flags >> 16);
    if (ntasks_left && (t.kind_dtype_flags & 0xffu) == kLaneGroup && seg < t.b)
        e = lanes[t.a + seg];
    return e;
}

template <int WAVES, int UL, int UC>
__global__ __launch_bounds__(WAVES * 64) void segmented_kernel(
    const uint8_t *__restrict__ base, const SegDesc *__restrict__ segs,
    const SegTask *__restrict__ tasks, uint32_t ntasks, uint32_t small_from,
    const SegLane *__restrict__ lanes, xsum_acc_t *states, SegCtl *ctl,
    int out_mode, uint64_t *out, uint32_t *flags)
{
    __shared__ WaveLds lds[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds &w = lds[wave];
    uint64_t *col = &w.cols[0][lane];
    zero_column<XSUM_F64>(col);

    // Items are claimed from the queue one at a time while they are large
    // (longest first is what balances the waves), and kSegPopBatch at a time
    // from item small_from on, where items are short.  The next claim is made
    // while the current one is handed out: a device-scope atomic's round trip
    // is long and its result is waited for where it is taken, so one wait
    // then serves several short items.
    uint32_t b0 = 0, n0 = 1, b1 = 0, n1 = 1, bi = 0;
    if (lane == 0) {
        b0 = atomicAdd(&ctl->head, 1u);
        b1 = atomicAdd(&ctl->head, 1u);
    }
    b0 = __shfl(b0, 0, 64);
    b1 = __shfl(b1, 0, 64);
    // next item index; each wave's indices only grow, so the first one past
    // the end ends the wave's work
    auto draw = [&]() -> uint32_t {
        if (bi == n0) {
            b0 = b1;
            n0 = n1;
            bi = 0;
            n1 = b0 >= small_from ? (uint32_t)kSegPopBatch : 1u;
            uint32_t claimed = 0;
            if (lane == 0)
                claimed = atomicAdd(&ctl->head, n1);
            b1 = __shfl(claimed, 0, 64);
        }
        return b0 + bi++;
    };

    // Work items flow through a three-stage pipeline so that no dependent
    // global access stands between two items: while item i runs, the record
    // and lane entry of item i + 1 and the record of item i + 2 are already
    // in registers or in flight.
    uint32_t cur = draw();
    uint32_t next = draw();
    uint32_t after = draw();
    SegTask t{}, nt{};
    if (cur < ntasks)
        t = tasks[cur];
    if (next < ntasks)
        nt = tasks[next];
    SegLane e = lane_entry(lanes, t, cur < ntasks, lane);
    while (cur < ntasks) {
        // issued before the item's own loads, consumed at the next item
        const SegLane ne = lane_entry(lanes, nt, next < ntasks, lane);
        SegTask nnt{};
        if (after < ntasks)
            nnt = tasks[after];
        const uint32_t following = draw();
        const uint32_t kind = t.kind_dtype_flags & 0xffu;
        const uint32_t dtype = (t.kind_dtype_flags >> 8) & 0xffu;
        if (kind == kLaneGroup) {
            const uint32_t glog = t.kind_dtype_flags >> 16;
            if (dtype == XSUM_F64)
                run_lane_group<XSUM_F64, UL>(base, e, t.b, glog, col, out_mode, out, flags,
                                              (const vec4u *)ctl->zero, lane);
            else if (dtype == XSUM_F32)
                run_lane_group<XSUM_F32, UL>(base, e, t.b, glog, col, out_mode, out, flags,
                                              (const vec4u *)ctl->zero, lane);
            else
                run_lane_group<XSUM_BF16, UL>(base, e, t.b, glog, col, out_mode, out, flags,
                                              (const vec4u *)ctl->zero, lane);
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
        cur = next;
        next = after;
        after = following;
        t = nt;
        nt = nnt;
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
                            const SegTask *tasks, uint32_t ntasks, uint32_t small_from,
                            const SegLane *lanes, xsum_acc_t *states,
                            SegCtl *ctl, int out_mode, uint64_t *out,
                            uint32_t *flags, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((segmented_kernel<kSegWaves, kSegLaneUnroll, kSegChunkUnroll>),
                       dim3((unsigned)blocks), dim3(kSegWaves * 64), 0, stream,
                       (const uint8_t *)base, segs, tasks, ntasks, small_from, lanes, states,
                       ctl, out_mode, out, flags);
    return hipGetLastError();
}

uint64_t segmented_chunk_vectors() { return 1ull << 16; }  // 1 MiB

}  // namespace xsum
