// Measurement kernels that carry none of the method: a plain streaming read
// with the launch shape of the binary64 single-sum kernel (the practical
// read ceiling that kernel is compared with), a buffer fill used to evict
// a working set from the caches between timed runs, and a sampler of the
// shader clock against the constant-rate clock, run beside timed launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "xsum.h"
#include "xsum_probe.h"

namespace xsum {
xsum_status_t api_fail(xsum_status_t st, const std::string &msg);
xsum_status_t api_hip_fail(hipError_t e, const char *what);
xsum_status_t api_current_cus(int *dev, int *cus);
}  // namespace xsum

namespace {

typedef uint32_t vec4u __attribute__((ext_vector_type(4)));

constexpr int kWaves = 2, kUnroll = 16, kBlocksPerCu = 2;
// the clock sampler runs for at most 10 s of the 100 MHz counter
constexpr uint32_t kClockMaxSamples = 1u << 20;
constexpr uint64_t kClockMaxTicks = 1000000000ull;

// Every wave streams its own run of 64 * kUnroll 16-byte vectors per tile
// with non-temporal loads, the next tile in flight while the current one is
// folded into an xor (the only arithmetic).  The xor is written out only if
// it equals a value that no caller's data is expected to give, so the loads
// stay live without a store per block.
__global__ __launch_bounds__(kWaves * 64) void read_probe_kernel(const vec4u *__restrict__ v,
                                                                 uint64_t nvec, uint32_t *sink)
{
    constexpr uint64_t kTile = (uint64_t)kWaves * 64 * kUnroll;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t my0 = (uint64_t)wave * 64 * kUnroll + lane;
    const uint64_t gstep = (uint64_t)gridDim.x * kTile;
    uint64_t tb = (uint64_t)blockIdx.x * kTile;
    uint32_t acc = 0;
    if (tb + kTile <= nvec) {
        vec4u qa[kUnroll], qb[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j)
            qa[j] = __builtin_nontemporal_load(v + tb + my0 + j * 64);
        for (;;) {
            uint64_t nb = tb + gstep;
            bool more = nb + kTile <= nvec;
            if (more) {
#pragma unroll
                for (int j = 0; j < kUnroll; ++j)
                    qb[j] = __builtin_nontemporal_load(v + nb + my0 + j * 64);
            }
#pragma unroll
            for (int j = 0; j < kUnroll; ++j)
                acc ^= qa[j].x ^ qa[j].y ^ qa[j].z ^ qa[j].w;
            tb = nb;
            if (!more)
                break;
            nb = tb + gstep;
            more = nb + kTile <= nvec;
            if (more) {
#pragma unroll
                for (int j = 0; j < kUnroll; ++j)
                    qa[j] = __builtin_nontemporal_load(v + nb + my0 + j * 64);
            }
#pragma unroll
            for (int j = 0; j < kUnroll; ++j)
                acc ^= qb[j].x ^ qb[j].y ^ qb[j].z ^ qb[j].w;
            tb = nb;
            if (!more)
                break;
        }
    }
    if (tb < nvec) {
        for (int j = 0; j < kUnroll; ++j) {
            const uint64_t i = tb + my0 + (uint64_t)j * 64;
            if (i < nvec) {
                const vec4u q = __builtin_nontemporal_load(v + i);
                acc ^= q.x ^ q.y ^ q.z ^ q.w;
            }
        }
    }
    if (acc == 0x9e3779b9u)
        sink[0] = acc;
}

__global__ void fill_kernel(uint32_t *p, uint64_t words, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// One lane takes nsamples samples, one every `interval` ticks of the
// 100 MHz constant-rate counter: that counter and the shader-clock counter,
// read back to back.  Every wait ends when the constant-rate counter passes
// its target, so the kernel runs for nsamples * interval ticks.
__global__ __launch_bounds__(64) void clock_probe_kernel(uint64_t *out, uint32_t nsamples,
                                                         uint32_t interval)
{
    if (threadIdx.x != 0)
        return;
    const uint64_t t0 = wall_clock64();
    for (uint32_t i = 0; i < nsamples; ++i) {
        const uint64_t target = t0 + (uint64_t)(i + 1) * interval;
        while (wall_clock64() < target) {
        }
        const uint64_t rt = wall_clock64();
        const uint64_t ck = clock64();
        out[2 * (uint64_t)i] = rt;
        out[2 * (uint64_t)i + 1] = ck;
    }
}

}  // namespace

extern "C" {

xsum_status_t xsum_probe_read(const void *x, uint64_t nbytes, uint32_t *sink, void *stream)
{
    if (nbytes == 0)
        return XSUM_OK;
    if (x == nullptr || sink == nullptr)
        return xsum::api_fail(XSUM_EINVAL, "x or sink is NULL");
    if ((uintptr_t)x % 16 != 0 || nbytes % 16 != 0)
        return xsum::api_fail(XSUM_EINVAL, "x and nbytes must be multiples of 16");
    int dev, cus;
    xsum_status_t st = xsum::api_current_cus(&dev, &cus);
    if (st != XSUM_OK)
        return st;
    const uint64_t nvec = nbytes / 16;
    const uint64_t tile = (uint64_t)kWaves * 64 * kUnroll;
    uint64_t blocks = (uint64_t)kBlocksPerCu * (uint64_t)cus;
    const uint64_t tiles = (nvec + tile - 1) / tile;
    if (blocks > tiles)
        blocks = tiles;
    hipLaunchKernelGGL(read_probe_kernel, dim3((unsigned)blocks), dim3(kWaves * 64), 0,
                       (hipStream_t)stream, (const vec4u *)x, nvec, sink);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? XSUM_OK : xsum::api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_probe_flush(void *buf, uint64_t nbytes, uint32_t value, void *stream)
{
    if (nbytes == 0)
        return XSUM_OK;
    if (buf == nullptr || (uintptr_t)buf % 4 != 0 || nbytes % 4 != 0)
        return xsum::api_fail(XSUM_EINVAL, "buf NULL, or buf / nbytes not multiples of 4");
    const uint64_t words = nbytes / 4;
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, (uint32_t *)buf, words, value);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? XSUM_OK : xsum::api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_probe_clock(uint64_t *out, uint32_t nsamples, uint32_t interval_ticks,
                               void *stream)
{
    if (nsamples == 0)
        return XSUM_OK;
    if (out == nullptr || (uintptr_t)out % 8 != 0)
        return xsum::api_fail(XSUM_EINVAL, "out is NULL or not 8-byte aligned");
    if (nsamples > kClockMaxSamples || interval_ticks == 0 ||
        (uint64_t)nsamples * interval_ticks > kClockMaxTicks)
        return xsum::api_fail(XSUM_ERANGE, "clock probe: nsamples <= 2^20, interval >= 1 tick, "
                                           "nsamples * interval <= 10 s");
    hipLaunchKernelGGL(clock_probe_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, out,
                       nsamples, interval_ticks);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? XSUM_OK : xsum::api_hip_fail(e, "kernel launch");
}

}  // extern "C"
