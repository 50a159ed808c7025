// Exact sums of inputs in host memory, streamed through the device (Section
// 5: when the superaccumulator fits in internal memory, one scan that adds
// the inputs in any order suffices; here the device state is the internal
// memory and the host array the external one, read once in chunks).
//
// Two device staging buffers alternate: while chunk c is added on the
// caller's stream, chunk c + 1 is copied host-to-device on a copy stream of
// the call's own.  Events order the two streams both ways (a buffer is
// refilled only after the kernel that read it has finished).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "xsum.h"
#include "xsum_internal.h"
#include "xsum_host.h"

namespace xsum {
xsum_status_t api_fail(xsum_status_t st, const std::string &msg);
xsum_status_t api_hip_fail(hipError_t e, const char *what);
xsum_status_t api_current_cus(int *dev, int *cus);
}  // namespace xsum

namespace {

using xsum::api_fail;
using xsum::api_hip_fail;

constexpr uint64_t kDefaultChunk = 64ull << 20;
constexpr uint64_t kMinChunk = 4096;
constexpr uint64_t kMaxChunk = 1ull << 34;

// Per-call resources, released on every exit path.
struct Staging {
    uint8_t *buf[2] = {nullptr, nullptr};
    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};
    hipEvent_t freed[2] = {nullptr, nullptr};

    ~Staging()
    {
        for (int b = 0; b < 2; ++b) {
            if (buf[b])
                (void)hipFree(buf[b]);
            if (copied[b])
                (void)hipEventDestroy(copied[b]);
            if (freed[b])
                (void)hipEventDestroy(freed[b]);
        }
        if (copy)
            (void)hipStreamDestroy(copy);
    }
};

xsum_status_t check_host_args(const void *x, uint64_t n, int dtype,
                              uint64_t chunk_bytes)
{
    if (dtype != XSUM_F64 && dtype != XSUM_F32 && dtype != XSUM_BF16)
        return api_fail(XSUM_EDTYPE, "unknown input dtype " + std::to_string(dtype));
    if (n > 0 && x == nullptr)
        return api_fail(XSUM_EINVAL, "host input pointer is NULL with n > 0");
    const int es = xsum::element_size(dtype);
    if ((uintptr_t)x % (uintptr_t)es != 0)
        return api_fail(XSUM_EINVAL, "host input pointer is not aligned to its element size");
    if (n > (UINT64_MAX >> 4))
        return api_fail(XSUM_ERANGE, "n too large");
    if (chunk_bytes != 0 &&
        (chunk_bytes < kMinChunk || chunk_bytes > kMaxChunk || chunk_bytes % 16 != 0))
        return api_fail(XSUM_ERANGE, "chunk_bytes must be 0 or a multiple of 16 in [4096, 2^34]");
    return XSUM_OK;
}

// acc += exact sum of the host array; returns once every chunk has been
// added (the caller's stream is synchronised).
xsum_status_t add_host(xsum_acc_t *acc, const void *x, uint64_t n, int dtype,
                       uint64_t chunk_bytes, hipStream_t s)
{
    if (n == 0)
        return XSUM_OK;
    int dev, cus;
    xsum_status_t st = xsum::api_current_cus(&dev, &cus);
    if (st != XSUM_OK)
        return st;
    const uint64_t es = (uint64_t)xsum::element_size(dtype);
    const uint64_t total = n * es;
    const uint64_t chunk = std::min(chunk_bytes ? chunk_bytes : kDefaultChunk,
                                    (total + 15) / 16 * 16);
    const uint64_t nchunks = (total + chunk - 1) / chunk;
    Staging sg;
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        if (b == 1 && nchunks < 2)
            break;
        e = hipMalloc((void **)&sg.buf[b], chunk);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&sg.copied[b], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&sg.freed[b], hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&sg.copy, hipStreamNonBlocking);
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? api_fail(XSUM_ENOMEM, "staging allocation failed")
                                        : api_hip_fail(e, "staging setup");
    const uint8_t *src = (const uint8_t *)x;
    const xsum::Finish keep{xsum::kKeep, XSUM_F64, nullptr, nullptr, 0};
    for (uint64_t c = 0; c < nchunks && e == hipSuccess; ++c) {
        const int b = (int)(c & 1);
        const uint64_t off = c * chunk;
        const uint64_t bytes = std::min(chunk, total - off);
        if (c >= 2)
            e = hipStreamWaitEvent(sg.copy, sg.freed[b], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sg.buf[b], src + off, bytes, hipMemcpyHostToDevice, sg.copy);
        if (e == hipSuccess)
            e = hipEventRecord(sg.copied[b], sg.copy);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, sg.copied[b], 0);
        if (e == hipSuccess)
            e = xsum::launch_accumulate(sg.buf[b], bytes / es, dtype, acc, keep, cus,
                                        xsum::Shape{0}, s);
        if (e == hipSuccess)
            e = hipEventRecord(sg.freed[b], s);
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(sg.copy);
        (void)hipStreamSynchronize(s);
        return api_hip_fail(e, "host streaming");
    }
    e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(sg.copy);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "hipStreamSynchronize");
}

}  // namespace

extern "C" {

xsum_status_t xsum_acc_add_host(xsum_acc_t *acc, const void *x_host, uint64_t n,
                                int dtype, uint64_t chunk_bytes, void *stream)
{
    if (acc == nullptr)
        return api_fail(XSUM_EINVAL, "acc is NULL");
    xsum_status_t st = check_host_args(x_host, n, dtype, chunk_bytes);
    if (st != XSUM_OK)
        return st;
    return add_host(acc, x_host, n, dtype, chunk_bytes, (hipStream_t)stream);
}

xsum_status_t xsum_exact_sum_host(const void *x_host, uint64_t n, int dtype,
                                  int out_dtype, void *out_host, uint32_t *flags_host,
                                  uint64_t chunk_bytes, void *stream)
{
    if (out_host == nullptr)
        return api_fail(XSUM_EINVAL, "out_host is NULL");
    xsum_status_t st = check_host_args(x_host, n, dtype, chunk_bytes);
    if (st != XSUM_OK)
        return st;
    const int of = xsum::resolve_out(dtype, out_dtype);
    if (of != XSUM_F64 && of != XSUM_F32 && of != XSUM_BF16)
        return api_fail(XSUM_EDTYPE, "unknown output dtype " + std::to_string(out_dtype));
    hipStream_t s = (hipStream_t)stream;
    xsum_acc_t *acc = nullptr;
    uint8_t *dev_out = nullptr;
    hipError_t e = hipMalloc((void **)&acc, sizeof(xsum_acc_t));
    if (e == hipSuccess)
        e = hipMalloc((void **)&dev_out, 16);
    if (e == hipSuccess)
        e = xsum::launch_zero(acc, 1, s);
    if (e != hipSuccess) {
        if (acc)
            (void)hipFree(acc);
        if (dev_out)
            (void)hipFree(dev_out);
        return e == hipErrorOutOfMemory ? api_fail(XSUM_ENOMEM, "state allocation failed")
                                        : api_hip_fail(e, "state setup");
    }
    st = add_host(acc, x_host, n, dtype, chunk_bytes, s);
    uint8_t host_out[16] = {0};
    if (st == XSUM_OK) {
        e = xsum::launch_finalize(acc, of, dev_out, (uint32_t *)(dev_out + 8), s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host_out, dev_out, 16, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            st = api_hip_fail(e, "finalize");
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(acc);
    (void)hipFree(dev_out);
    if (st != XSUM_OK)
        return st;
    std::memcpy(out_host, host_out, (size_t)xsum::out_bytes(of));
    if (flags_host)
        std::memcpy(flags_host, host_out + 8, 4);
    return XSUM_OK;
}

}  // extern "C"
