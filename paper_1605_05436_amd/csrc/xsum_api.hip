// C-ABI entry points of libxsum: argument checks, per-(device, stream)
// workspaces for the blocking call, and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "xsum.h"
#include "xsum_internal.h"
#include "xsum_host.h"

namespace {

thread_local std::string g_err;

xsum_status_t fail(xsum_status_t st, const std::string &msg)
{
    g_err = msg;
    return st;
}

xsum_status_t hip_fail(hipError_t e, const char *what)
{
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s (hipError %d)", what,
                  hipGetErrorString(e), (int)e);
    g_err = buf;
    return XSUM_EHIP;
}

std::mutex g_mu;
std::map<int, int> g_cu_count;

// Workspace of the blocking call for one (device, stream): a zeroed scratch
// state (left zeroed by every completed call), a device result slot and a
// pinned host slot for the copy back.
struct BlockingWs {
    xsum_acc_t *acc = nullptr;
    uint8_t *dev_out = nullptr;   // 8 bytes result + 4 bytes flags
    uint8_t *host_out = nullptr;  // pinned, 16 bytes
    std::mutex mu;                // orders calls on the same stream
};
std::map<std::pair<int, void *>, BlockingWs *> g_ws;

bool valid_in(int d) { return d == XSUM_F64 || d == XSUM_F32 || d == XSUM_BF16; }

using xsum::out_bytes;
using xsum::resolve_out;

xsum_status_t check_input(const void *x, uint64_t n, int dtype)
{
    if (!valid_in(dtype))
        return fail(XSUM_EDTYPE, "unknown input dtype " + std::to_string(dtype));
    if (n > 0 && x == nullptr)
        return fail(XSUM_EINVAL, "input pointer is NULL with n > 0");
    const int es = xsum::element_size(dtype);
    if ((uintptr_t)x % (uintptr_t)es != 0)
        return fail(XSUM_EINVAL, "input pointer is not aligned to its element size");
    if (n > (UINT64_MAX >> 4))
        return fail(XSUM_ERANGE, "n too large");
    return XSUM_OK;
}

xsum_status_t current_cus(int *dev, int *cus)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cu_count.find(*dev);
    if (it != g_cu_count.end()) {
        *cus = it->second;
        return XSUM_OK;
    }
    int c = 0;
    e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, *dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    if (c < 1)
        c = 1;
    g_cu_count[*dev] = c;
    *cus = c;
    return XSUM_OK;
}

xsum_status_t blocking_ws(int dev, void *stream, BlockingWs **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return XSUM_OK;
    }
    BlockingWs *w = new BlockingWs();
    hipError_t e = hipMalloc((void **)&w->acc, sizeof(xsum_acc_t));
    if (e == hipSuccess)
        e = hipMalloc((void **)&w->dev_out, 16);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&w->host_out, 16, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipMemset(w->acc, 0, sizeof(xsum_acc_t));
    if (e != hipSuccess) {
        if (w->acc)
            (void)hipFree(w->acc);
        if (w->dev_out)
            (void)hipFree(w->dev_out);
        if (w->host_out)
            (void)hipHostFree(w->host_out);
        delete w;
        return e == hipErrorOutOfMemory ? fail(XSUM_ENOMEM, "workspace allocation failed")
                                        : hip_fail(e, "workspace allocation");
    }
    g_ws[key] = w;
    *out = w;
    return XSUM_OK;
}

xsum_status_t sum_async(const void *x, uint64_t n, int dtype, int out_dtype,
                        void *out_dev, uint32_t *flags_dev,
                        xsum_acc_t *scratch, void *stream, int blocks)
{
    xsum_status_t st = check_input(x, n, dtype);
    if (st != XSUM_OK)
        return st;
    const int of = resolve_out(dtype, out_dtype);
    if (!valid_in(of))
        return fail(XSUM_EDTYPE, "unknown output dtype " + std::to_string(out_dtype));
    if (out_dev == nullptr || scratch == nullptr)
        return fail(XSUM_EINVAL, "output or scratch pointer is NULL");
    if (blocks < 0)
        return fail(XSUM_EINVAL, "negative block count");
    int dev, cus;
    if ((st = current_cus(&dev, &cus)) != XSUM_OK)
        return st;
    xsum::Finish fin{xsum::kRound, of, out_dev, flags_dev, 0};
    hipError_t e = xsum::launch_accumulate(x, n, dtype, scratch, fin, cus,
                                           xsum::Shape{blocks},
                                           (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "kernel launch");
    return XSUM_OK;
}

}  // namespace

namespace xsum {
xsum_status_t api_fail(xsum_status_t st, const std::string &msg) { return fail(st, msg); }
xsum_status_t api_hip_fail(hipError_t e, const char *what) { return hip_fail(e, what); }
xsum_status_t api_current_cus(int *dev, int *cus) { return current_cus(dev, cus); }
}  // namespace xsum

extern "C" {

const char *xsum_version(void) { return "xsum 0.1.0 gfx950"; }

const char *xsum_last_error(void) { return g_err.c_str(); }

xsum_status_t xsum_exact_sum_async(const void *x, uint64_t n, int dtype,
                                   int out_dtype, void *out_dev,
                                   uint32_t *flags_dev, xsum_acc_t *scratch,
                                   void *stream)
{
    return sum_async(x, n, dtype, out_dtype, out_dev, flags_dev, scratch,
                     stream, 0);
}

xsum_status_t xsum_exact_sum_async_blocks(const void *x, uint64_t n,
                                          int dtype, int out_dtype,
                                          void *out_dev, uint32_t *flags_dev,
                                          xsum_acc_t *scratch, int blocks,
                                          void *stream)
{
    return sum_async(x, n, dtype, out_dtype, out_dev, flags_dev, scratch,
                     stream, blocks);
}

xsum_status_t xsum_exact_sum(const void *x, uint64_t n, int dtype,
                             int out_dtype, void *out_host,
                             uint32_t *flags_host, void *stream)
{
    if (out_host == nullptr)
        return fail(XSUM_EINVAL, "out_host is NULL");
    xsum_status_t st = check_input(x, n, dtype);
    if (st != XSUM_OK)
        return st;
    const int of = resolve_out(dtype, out_dtype);
    if (!valid_in(of))
        return fail(XSUM_EDTYPE, "unknown output dtype " + std::to_string(out_dtype));
    int dev, cus;
    if ((st = current_cus(&dev, &cus)) != XSUM_OK)
        return st;
    BlockingWs *w;
    if ((st = blocking_ws(dev, stream, &w)) != XSUM_OK)
        return st;
    std::lock_guard<std::mutex> lk(w->mu);
    xsum::Finish fin{xsum::kRound, of, w->dev_out, (uint32_t *)(w->dev_out + 8), 0};
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = xsum::launch_accumulate(x, n, dtype, w->acc, fin, cus,
                                           xsum::Shape{0}, s);
    if (e != hipSuccess)
        return hip_fail(e, "kernel launch");
    e = hipMemcpyAsync(w->host_out, w->dev_out, 16, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamSynchronize");
    std::memcpy(out_host, w->host_out, (size_t)out_bytes(of));
    if (flags_host)
        std::memcpy(flags_host, w->host_out + 8, 4);
    return XSUM_OK;
}

double xsum_exact_sum_f64(const void *x, uint64_t n, int dtype)
{
    double r;
    if (xsum_exact_sum(x, n, dtype, XSUM_F64, &r, nullptr, nullptr) != XSUM_OK)
        return __builtin_nan("");
    return r;
}

xsum_status_t xsum_acc_zero(xsum_acc_t *acc, uint64_t count, void *stream)
{
    if (count == 0)
        return XSUM_OK;
    if (acc == nullptr)
        return fail(XSUM_EINVAL, "acc is NULL");
    hipError_t e = xsum::launch_zero(acc, count, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : hip_fail(e, "kernel launch");
}

xsum_status_t xsum_acc_add(xsum_acc_t *acc, const void *x, uint64_t n,
                           int dtype, void *stream)
{
    if (acc == nullptr)
        return fail(XSUM_EINVAL, "acc is NULL");
    xsum_status_t st = check_input(x, n, dtype);
    if (st != XSUM_OK)
        return st;
    int dev, cus;
    if ((st = current_cus(&dev, &cus)) != XSUM_OK)
        return st;
    xsum::Finish fin{xsum::kKeep, XSUM_F64, nullptr, nullptr, 0};
    hipError_t e = xsum::launch_accumulate(x, n, dtype, acc, fin, cus,
                                           xsum::Shape{0}, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : hip_fail(e, "kernel launch");
}

xsum_status_t xsum_acc_merge(xsum_acc_t *dst, const xsum_acc_t *src,
                             void *stream)
{
    if (dst == nullptr || src == nullptr)
        return fail(XSUM_EINVAL, "dst or src is NULL");
    hipError_t e = xsum::launch_merge(dst, src, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : hip_fail(e, "kernel launch");
}

xsum_status_t xsum_acc_finalize(const xsum_acc_t *acc, int out_dtype,
                                void *out_dev, uint32_t *flags_dev,
                                void *stream)
{
    if (acc == nullptr || out_dev == nullptr)
        return fail(XSUM_EINVAL, "acc or out is NULL");
    const int of = out_dtype == XSUM_SAME ? XSUM_F64 : out_dtype;
    if (!valid_in(of))
        return fail(XSUM_EDTYPE, "unknown output dtype " + std::to_string(out_dtype));
    hipError_t e = xsum::launch_finalize(acc, of, out_dev, flags_dev,
                                         (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : hip_fail(e, "kernel launch");
}

}  // extern "C"
