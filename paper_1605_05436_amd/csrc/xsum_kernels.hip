// Single exact sum and accumulator-state kernels for gfx950 (CDNA4).
//
// One launch computes one exact sum (Section 3 steps 2, 5, 6, 7 of Goodrich &
// Eldawy; Section 5's scan algorithm, whose whole accumulator fits in fast
// memory; Section 6's combine / reduce / post-process structure):
//   1. load      128-bit non-temporal loads, grid-stride over 16-byte vectors,
//                software-pipelined (the next tile is in flight while the
//                current one is added)
//   2. split     decode each element and cut its shifted significand into
//                chunks at digit (or bin) boundaries
//   3. add       chunks go to the lane's private LDS column, carry-free
//   4. block     the wave's 64 columns are summed per digit with one local
//                carry split; the block's non-zero digits go to the global
//                state with int64 atomics
//   5. ticket    the last block to finish takes over the global state
//   6. normalise two local carry steps bring every digit to [-1, 2^32]; a
//                wave-wide prefix over the carry transfer functions
//                {-1,0,1} -> {-1,0,1} (the paper's lookup-table prefix) gives
//                canonical digits and the sign
//   7. round     the top non-zero digit, its two neighbours and a sticky bit
//                give the round-to-nearest-even result
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xsum.h"
#include "xsum_device.h"
#include "xsum_internal.h"

namespace xsum {

// x: first element; head elements precede the 16-byte-aligned vector part
// of nvec 16-byte vectors, followed by tail elements.
//
// binary64 columns are carry-normalised after every pair of full tiles that
// brings the count of tiles since the last normalisation to kNormTiles or
// more.  Between two normalisations a column therefore receives at most
// (kNormTiles + 1) full tiles, one partial tile and a head/tail element,
// fewer than (kNormTiles + 2)*U*2 + 2 < 2047 elements, each adding below
// 2^32 + 2^52 to a digit that started below 2^32: every entry stays below
// 2^63 and its high word below 2^31 in magnitude, as the block merge assumes.
// Binned (binary32, bfloat16) entries only grow.  binary32: the launcher
// gives every block at most 2^24 tiles of U * kPerVec = 64 elements per lane,
// each chunk below 2^31, so an entry stays below 2^61 and its high word below
// 2^31, as the block merge assumes.  bfloat16 entries are 32-bit (half the
// LDS, so twice the resident waves): chunks are below 2^15, and every
// kFlushTiles tiles each wave merges its columns into the block vector and
// clears them, so an entry receives fewer than (kFlushTiles + 2) * U * 8 + 2
// < 2^17 chunks between clears.
template <int FMT, int WAVES, int U, bool WAVE_CONTIG>
__global__ __launch_bounds__(WAVES * 64) void accumulate_kernel(
    const uint8_t *__restrict__ x, uint32_t head, uint64_t nvec,
    uint32_t tail, xsum_acc_t *acc, Finish fin)
{
    using G = Geo<FMT>;
    constexpr int kThreads = WAVES * 64;
    constexpr uint64_t kTile = (uint64_t)kThreads * U;  // vectors per block step
    constexpr int kNormTiles = 512 / U;
    static_assert(FMT != XSUM_F64 || (kNormTiles + 2) * U * 2 + 2 < 2047,
                  "binary64 column headroom");
    constexpr int kFlushTiles = 256;
    static_assert(FMT != XSUM_F32 || U * 4 <= 64, "binary32 column headroom");
    static_assert(FMT != XSUM_BF16 || (kFlushTiles + 2) * U * 8 + 2 < (1 << 17),
                  "bfloat16 column headroom");
    using ColT = std::conditional_t<FMT == XSUM_BF16, uint32_t, uint64_t>;
    __shared__ ColT cols[WAVES][G::kN][64];
    __shared__ int64_t blk[kDigits];
    __shared__ uint32_t blk_spec;
    __shared__ int is_last;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    ColT *col = &cols[wave][0][lane];
    // vector j of this thread within a tile: interleaved across the block, or
    // a contiguous 64*U-vector run per wave
    const uint64_t my0 = WAVE_CONTIG ? (uint64_t)wave * 64 * U + lane : (uint64_t)tid;
    constexpr uint64_t kJStride = WAVE_CONTIG ? 64 : kThreads;
#pragma unroll
    for (int d = 0; d < G::kN; ++d)
        col[d * 64] = 0;
    for (int d = tid; d < kDigits; d += kThreads)
        blk[d] = 0;
    if (tid == 0)
        blk_spec = 0;
    __syncthreads();    // blk is zero before any wave flushes into it
    uint32_t spec = 0;

    const vec4u *v = (const vec4u *)(x + (uint64_t)head * G::kBytes);
    const uint64_t gstep = (uint64_t)gridDim.x * kTile;
    uint64_t tb = (uint64_t)blockIdx.x * kTile;
    int since_norm = 0;

    if (tb + kTile <= nvec) {
        vec4u qa[U], qb[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            qa[j] = __builtin_nontemporal_load(v + tb + my0 + j * kJStride);
        for (;;) {
            uint64_t nb = tb + gstep;
            bool more = nb + kTile <= nvec;
            if (more) {
#pragma unroll
                for (int j = 0; j < U; ++j)
                    qb[j] = __builtin_nontemporal_load(v + nb + my0 + j * kJStride);
            }
            add_tile<FMT, U>(qa, col, spec);
            tb = nb;
            if (!more)
                break;
            nb = tb + gstep;
            more = nb + kTile <= nvec;
            if (more) {
#pragma unroll
                for (int j = 0; j < U; ++j)
                    qa[j] = __builtin_nontemporal_load(v + nb + my0 + j * kJStride);
            }
            add_tile<FMT, U>(qb, col, spec);
            tb = nb;
            if constexpr (FMT == XSUM_F64) {
                since_norm += 2;
                if (since_norm >= kNormTiles) {
                    normalise_column<G::kN>(col);
                    since_norm = 0;
                }
            } else if constexpr (FMT == XSUM_BF16) {
                since_norm += 2;
                if (since_norm >= kFlushTiles) {
                    wave_lds_fence();
                    merge_wave_columns<FMT>(cols[wave], blk, lane);
                    wave_lds_fence();
#pragma unroll
                    for (int d = 0; d < G::kN; ++d)
                        col[d * 64] = 0;
                    since_norm = 0;
                }
            }
            if (!more)
                break;
        }
    }
    // At most one partial tile exists (the last); its owner finishes it.
    if (tb < nvec) {
        for (int j = 0; j < U; ++j) {
            const uint64_t i = tb + my0 + (uint64_t)j * kJStride;
            vec4u q[1] = {{0u, 0u, 0u, 0u}};
            if (i < nvec)
                q[0] = __builtin_nontemporal_load(v + i);
            add_tile<FMT, 1>(q, col, spec);
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

    merge_wave_columns<FMT>(cols[wave], blk, lane);
    if (spec)
        __hip_atomic_fetch_or(&blk_spec, spec, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();

    // Grid merge: add the block's non-zero digits into the global state.
    // Every access to the state is a system-scope atomic read-modify-write,
    // performed at the memory side past every XCD's L2, so publishing needs
    // no L2 write-back: each block only waits until its own atomics have
    // completed before it takes its ticket (an agent-scope release fence
    // would write back the XCD's whole L2 once per block while the other
    // blocks still stream, which costs several percent of a large sum).
    for (int d = tid; d < kDigits; d += kThreads) {
        const int64_t dv = blk[d];
        if (dv)
            __hip_atomic_fetch_add(&acc->digit[d], dv, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (tid == 0 && blk_spec)
        __hip_atomic_fetch_or(&acc->special, blk_spec, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
    // the fence keeps the atomics above this point; the wait (every counter
    // zero) returns once they have completed at the memory side
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
        const unsigned t = __hip_atomic_fetch_add(&acc->ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last)
        return;
    if (wave == 0)
        finish_state<true>(acc, fin, lane);
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

// Launch shapes (measured on MI355X with the timing harness, config-2-like
// data): a column is 66 x 64 x 8 B = 33 KiB per wave for binary64 and
// binary32, so four waves fill a CU's 160 KiB of LDS; bfloat16's 32-bit
// entries take half that, so eight one-wave blocks fit (two waves per SIMD).
// Each wave keeps U 16-byte loads per lane in flight while it adds the
// previous U; wave-contiguous tiles give each wave its own 64*U-vector
// stream.
template <int FMT> struct Shape_;
template <> struct Shape_<XSUM_F64> {
    static constexpr int kWaves = 2, kUnroll = 16, kBlocksPerCu = 2;
    static constexpr bool kWaveContig = true;
};
template <> struct Shape_<XSUM_F32> {
    static constexpr int kWaves = 2, kUnroll = 16, kBlocksPerCu = 2;
    static constexpr bool kWaveContig = true;
};
template <> struct Shape_<XSUM_BF16> {
    static constexpr int kWaves = 1, kUnroll = 24, kBlocksPerCu = 8;
    static constexpr bool kWaveContig = true;
};

int persistent_blocks(int dtype, int cu_count)
{
    switch (dtype) {
    case XSUM_F64:
        return Shape_<XSUM_F64>::kBlocksPerCu * cu_count;
    case XSUM_F32:
        return Shape_<XSUM_F32>::kBlocksPerCu * cu_count;
    default:
        return Shape_<XSUM_BF16>::kBlocksPerCu * cu_count;
    }
}

template <int FMT>
static hipError_t launch_fmt(const void *x, uint64_t n, xsum_acc_t *acc,
                             const Finish &fin, int cu_count,
                             const Shape &shape, hipStream_t stream)
{
    using G = Geo<FMT>;
    using S = Shape_<FMT>;
    const uintptr_t addr = (uintptr_t)x;
    uint64_t head = ((16 - (addr & 15)) & 15) / G::kBytes;
    if (head > n)
        head = n;
    const uint64_t rest = n - head;
    const uint64_t nvec = rest / G::kPerVec;
    const uint64_t tail = rest - nvec * G::kPerVec;
    const uint64_t tile = (uint64_t)S::kWaves * 64 * S::kUnroll;
    const uint64_t tiles = (nvec + tile - 1) / tile;
    uint64_t blocks;
    if (shape.blocks > 0) {
        blocks = (uint64_t)shape.blocks;
    } else {
        // Every block pays a fixed merge, its grid atomics and a ticket, so
        // a small input gets about one block per 16 KiB (at least 32 blocks
        // to keep the loads spread), a large one the persistent grid.
        constexpr uint64_t kVectorsPerBlock = 1024, kMinBlocks = 32;
        blocks = (uint64_t)persistent_blocks(FMT, cu_count);
        const uint64_t want = (nvec + kVectorsPerBlock - 1) / kVectorsPerBlock;
        if (want < blocks)
            blocks = want > kMinBlocks ? want : kMinBlocks;
    }
    constexpr uint64_t kMaxTilesPerBlock = uint64_t(1) << 24;
    if (blocks < (tiles + kMaxTilesPerBlock - 1) / kMaxTilesPerBlock)
        blocks = (tiles + kMaxTilesPerBlock - 1) / kMaxTilesPerBlock;
    if (blocks > tiles)
        blocks = tiles;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL((accumulate_kernel<FMT, S::kWaves, S::kUnroll, S::kWaveContig>),
                       dim3((unsigned)blocks), dim3(S::kWaves * 64), 0, stream,
                       (const uint8_t *)x, (uint32_t)head, nvec, (uint32_t)tail, acc, fin);
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
    return launch_zero_words((uint64_t *)acc, count * (sizeof(xsum_acc_t) / 8), stream);
}

hipError_t launch_zero_words(uint64_t *p, uint64_t words, hipStream_t stream)
{
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       p, words);
    return hipGetLastError();
}

}  // namespace xsum
