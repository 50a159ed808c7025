// Segmented exact sums: many independent sums, of uneven lengths and mixed
// formats, in one persistent launch (Section 6 of Goodrich & Eldawy: every
// reducer sums its own numbers into a superaccumulator; long inputs are first
// combined per chunk and the per-chunk states merged and rounded once).
//
// Work items come from a host-built plan, popped by every wave from a shared
// queue (one device atomic per item):
//   * lane group: up to 64 whole segments of one format and similar length
//     (the plan sorts segments by length).  Each lane streams its own segment
//     into its private LDS column exactly as the single-sum kernel does, then
//     carry-normalises and rounds it alone (LaneFinisher), so a segment costs
//     about 1/64 of a wave's fixed work.
//   * chunk: a contiguous run of one long segment, loaded coalesced by a whole
//     wave.  The wave merges its 64 columns and adds the digits into the
//     segment's state with int64 atomics; a per-segment ticket lets the last
//     chunk round the state (and zero it for the next launch).
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

// Per-wave LDS: a binary64-sized column set (binary32 tasks use the first
// 33 entries) and a 68-digit merge vector.
struct WaveLds {
    uint64_t cols[Geo<XSUM_F64>::kN][64];
    int64_t merged[kDigits];
};

__device__ __forceinline__ void wave_lds_fence()
{
    // every LDS operation of this wave issued so far has completed and is
    // ordered before what follows (other lanes' column entries are read next)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

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
// 0..65; binary32 bins (weight 2^(8(b + 115))) are first moved to radix-2^32
// digits 28..38 (each bin split into 32-bit halves so no shift overflows).
template <int FMT>
__device__ __forceinline__ uint64_t finish_lane(uint64_t *col, uint32_t spec,
                                                int out_fmt, uint32_t &flags)
{
    LaneFinisher fin;
    if constexpr (FMT == XSUM_F64) {
#pragma unroll
        for (int d = 0; d < Geo<XSUM_F64>::kN; ++d) {
            fin.feed((int64_t)lds_load(col + d * 64));
            lds_store(col + d * 64, 0);
        }
        return fin.round(spec, out_fmt, 0, flags);
    } else {
        constexpr int kD = 11;           // digits 28..38
        int64_t dig[kD];
#pragma unroll
        for (int i = 0; i < kD; ++i)
            dig[i] = 0;
#pragma unroll
        for (int b = 0; b < Geo<FMT>::kN; ++b) {
            const int64_t v = (int64_t)lds_load(col + b * 64);
            lds_store(col + b * 64, 0);
            const int g = ((b + Geo<FMT>::kBin0) >> 2) - 28;
            const int sh = 8 * ((b + Geo<FMT>::kBin0) & 3);
            const uint64_t lo = ((uint64_t)v & kLow32) << sh;     // < 2^56
            const int64_t hi = (int64_t)((uint64_t)(v >> 32) << sh);
            dig[g] += (int64_t)(lo & kLow32);
            dig[g + 1] += (int64_t)(lo >> 32) + hi;
        }
#pragma unroll
        for (int i = 0; i < kD; ++i)
            fin.feed(dig[i]);
        return fin.round(spec, out_fmt, 28, flags);
    }
}

// One lane group: lane l < count sums segment perm[first + l].
template <int FMT, int UL>
__device__ void run_lane_group(const uint8_t *base, const SegDesc *segs,
                               const uint32_t *perm, uint32_t first,
                               uint32_t count, uint64_t *col, int out_mode,
                               uint64_t *out, uint32_t *flags, int lane)
{
    using G = Geo<FMT>;
    const bool live = (uint32_t)lane < count;
    uint32_t s = 0;
    uint64_t L = 0, off = 0;
    if (live) {
        s = perm[first + lane];
        off = segs[s].byte_offset;
        L = segs[s].length;
    }
    const uint8_t *p = base + off;
    uint64_t head = ((16 - ((uintptr_t)p & 15)) & 15) / G::kBytes;
    if (head > L)
        head = L;
    const uint64_t nv = (L - head) / G::kPerVec;
    const uint64_t tail = L - head - nv * G::kPerVec;
    const vec4u *vp = (const vec4u *)(p + head * G::kBytes);
    uint32_t spec = 0;

    const uint64_t my_iters = (nv + UL - 1) / UL;
    const uint32_t iters = wave_max_u32((uint32_t)my_iters);
    constexpr int kNormIters = 512 / UL;   // binary64: <= 1024 + 2*UL + 14 elements between normalisations
    int since = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        vec4u q[UL];
#pragma unroll
        for (int j = 0; j < UL; ++j) {
            const uint64_t i = (uint64_t)it * UL + j;
            q[j] = vec4u{0u, 0u, 0u, 0u};
            if (i < nv)
                q[j] = __builtin_nontemporal_load(vp + i);
        }
        add_tile<FMT, UL>(q, col, spec);
        if constexpr (FMT == XSUM_F64) {
            if (++since >= kNormIters) {
                normalise_column<G::kN>(col);
                since = 0;
            }
        }
    }
    for (uint64_t i = 0; i < head; ++i)
        add_scalar<FMT>(p + i * G::kBytes, col, spec);
    const uint8_t *tp = p + head * G::kBytes + nv * 16;
    for (uint64_t i = 0; i < tail; ++i)
        add_scalar<FMT>(tp + i * G::kBytes, col, spec);

    const int of = out_mode == XSUM_SAME ? LaneOut<FMT>::kNatural : out_mode;
    uint32_t fl;
    const uint64_t bits = finish_lane<FMT>(col, spec, of, fl);
    if (live) {
        out[s] = bits;
        if (flags)
            flags[s] = fl;
    }
}

// One chunk of a long segment, summed by the whole wave.
template <int FMT, int UC>
__device__ void run_chunk(const uint8_t *base, const SegDesc *segs,
                          const SegTask &t, xsum_acc_t *states, WaveLds &w,
                          uint64_t *col, int out_mode, uint64_t *out,
                          uint32_t *flags, int lane)
{
    using G = Geo<FMT>;
    const uint32_t s = t.a;
    const uint32_t cflags = t.kind_dtype_flags >> 16;
    const uint8_t *p = base + segs[s].byte_offset;
    const uint64_t L = segs[s].length;
    uint64_t head = ((16 - ((uintptr_t)p & 15)) & 15) / G::kBytes;
    if (head > L)
        head = L;
    const uint64_t nvs = (L - head) / G::kPerVec;
    const uint64_t tail = L - head - nvs * G::kPerVec;
    const vec4u *vp = (const vec4u *)(p + head * G::kBytes) + t.v0;
    const uint64_t nv = t.nv;
    uint32_t spec = 0;

    // wave-contiguous tiles of 64*UC vectors, next tile in flight
    constexpr uint64_t kTile = 64ull * UC;
    constexpr int kNormTiles = 512 / UC;
    const uint64_t full = nv / kTile;
    int since = 0;
    if (full > 0) {
        vec4u qa[UC], qb[UC];
#pragma unroll
        for (int j = 0; j < UC; ++j)
            qa[j] = __builtin_nontemporal_load(vp + j * 64 + lane);
        for (uint64_t tt = 0; tt < full; tt += 2) {
            const bool more_b = tt + 1 < full;
            if (more_b) {
#pragma unroll
                for (int j = 0; j < UC; ++j)
                    qb[j] = __builtin_nontemporal_load(vp + (tt + 1) * kTile + j * 64 + lane);
            }
            add_tile<FMT, UC>(qa, col, spec);
            if (!more_b)
                break;
            const bool more_a = tt + 2 < full;
            if (more_a) {
#pragma unroll
                for (int j = 0; j < UC; ++j)
                    qa[j] = __builtin_nontemporal_load(vp + (tt + 2) * kTile + j * 64 + lane);
            }
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
    for (uint64_t i = full * kTile + lane; i < nv; i += 64) {
        vec4u q[1] = {__builtin_nontemporal_load(vp + i)};
        add_tile<FMT, 1>(q, col, spec);
    }
    if ((cflags & kChunkFirst) && (uint64_t)lane < head)
        add_scalar<FMT>(p + (uint64_t)lane * G::kBytes, col, spec);
    if ((cflags & kChunkLast) && (uint64_t)lane < tail)
        add_scalar<FMT>(p + head * G::kBytes + nvs * 16 + (uint64_t)lane * G::kBytes,
                        col, spec);

    // merge the wave's columns, then clear them for the next item
    for (int d = lane; d < kDigits; d += 64)
        w.merged[d] = 0;
    wave_lds_fence();
    merge_wave_columns<FMT>(w.cols, w.merged, lane);
    wave_lds_fence();
    zero_column<FMT>(col);
    spec = wave_or_u32(spec);

    xsum_acc_t *st = &states[t.b];
    for (int d = lane; d < kDigits; d += 64) {
        const int64_t dv = w.merged[d];
        if (dv)
            atomicAdd((unsigned long long *)&st->digit[d], (unsigned long long)dv);
    }
    if (lane == 0 && spec)
        atomicOr(&st->special, spec);
    __threadfence();
    uint32_t ticket = 0;
    if (lane == 0)
        ticket = atomicAdd(&st->ticket, 1u);
    ticket = __shfl(ticket, 0, 64);
    if (ticket == t.nchunks - 1) {
        __threadfence();
        const int of = out_mode == XSUM_SAME ? LaneOut<FMT>::kNatural : out_mode;
        Finish fin{kRound, of, out + s, flags ? flags + s : nullptr, 1};
        finish_state(st, fin, lane);
    }
}

template <int WAVES, int UL, int UC>
__global__ __launch_bounds__(WAVES * 64) void segmented_kernel(
    const uint8_t *__restrict__ base, const SegDesc *__restrict__ segs,
    const SegTask *__restrict__ tasks, uint32_t ntasks,
    const uint32_t *__restrict__ perm, xsum_acc_t *states, SegCtl *ctl,
    int out_mode, uint64_t *out, uint32_t *flags)
{
    __shared__ WaveLds lds[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds &w = lds[wave];
    uint64_t *col = &w.cols[0][lane];
    zero_column<XSUM_F64>(col);

    for (;;) {
        uint32_t ti = 0;
        if (lane == 0)
            ti = atomicAdd(&ctl->head, 1u);
        ti = __shfl(ti, 0, 64);
        if (ti >= ntasks)
            break;
        const SegTask t = tasks[ti];
        const uint32_t kind = t.kind_dtype_flags & 0xffu;
        const uint32_t dtype = (t.kind_dtype_flags >> 8) & 0xffu;
        if (kind == kLaneGroup) {
            if (dtype == XSUM_F64)
                run_lane_group<XSUM_F64, UL>(base, segs, perm, t.a, t.b, col, out_mode, out, flags, lane);
            else if (dtype == XSUM_F32)
                run_lane_group<XSUM_F32, UL>(base, segs, perm, t.a, t.b, col, out_mode, out, flags, lane);
            else
                run_lane_group<XSUM_BF16, UL>(base, segs, perm, t.a, t.b, col, out_mode, out, flags, lane);
        } else {
            if (dtype == XSUM_F64)
                run_chunk<XSUM_F64, UC>(base, segs, t, states, w, col, out_mode, out, flags, lane);
            else if (dtype == XSUM_F32)
                run_chunk<XSUM_F32, UC>(base, segs, t, states, w, col, out_mode, out, flags, lane);
            else
                run_chunk<XSUM_BF16, UC>(base, segs, t, states, w, col, out_mode, out, flags, lane);
        }
    }
    // the last wave out resets the queue for the next launch
    if (lane == 0) {
        __threadfence();
        const uint32_t total = gridDim.x * WAVES;
        if (atomicAdd(&ctl->done, 1u) == total - 1) {
            __hip_atomic_store(&ctl->head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

static constexpr int kSegWaves = 1;
static constexpr int kSegLaneUnroll = 4;
static constexpr int kSegChunkUnroll = 16;
static constexpr int kSegBlocksPerCu = 4;

int segmented_blocks(int cu_count, int blocks_per_cu)
{
    return (blocks_per_cu > 0 ? blocks_per_cu : kSegBlocksPerCu) * cu_count;
}

hipError_t launch_segmented(const void *base, const SegDesc *segs,
                            const SegTask *tasks, uint32_t ntasks,
                            const uint32_t *perm, xsum_acc_t *states,
                            SegCtl *ctl, int out_mode, uint64_t *out,
                            uint32_t *flags, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((segmented_kernel<kSegWaves, kSegLaneUnroll, kSegChunkUnroll>),
                       dim3((unsigned)blocks), dim3(kSegWaves * 64), 0, stream,
                       (const uint8_t *)base, segs, tasks, ntasks, perm, states,
                       ctl, out_mode, out, flags);
    return hipGetLastError();
}

uint64_t segmented_chunk_vectors() { return 64ull * kSegChunkUnroll * 8; }

}  // namespace xsum
