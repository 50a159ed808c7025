// Compact encoding of an exact state for checkpoints and exchange (host code
// only).  Section 2 keeps a superaccumulator sparse: only its non-zero
// components are stored, each with its exponent.  Here the state is first
// carry-normalised (Section 3, step 6: signed carry propagation) and its
// magnitude is stored as the one contiguous run of radix-2^32 digits from the
// lowest to the highest non-zero digit, with the run's starting index, the
// sign and the special-value bits.
#include <cstdint>
#include <cstring>
#include <string>

#include "xsum.h"

namespace xsum {
xsum_status_t api_fail(xsum_status_t st, const std::string &msg);
}  // namespace xsum

namespace {

constexpr uint32_t kMagic = 0x31535358u;   // "XSS1"
constexpr int kWide = 70;                   // digits of the two's-complement value
constexpr int kHeader = 12;
constexpr int64_t kDigitLimit = int64_t(1) << 62;
constexpr int64_t kTopLimit = int64_t(1) << 61;   // normalised top digit

// Two's complement of the state's value over kWide radix-2^32 digits.
// Every input digit must satisfy |d| <= 2^62 so no step overflows.
void to_wide(const xsum_acc_t &acc, uint32_t w[kWide])
{
    int64_t carry = 0;
    for (int j = 0; j < XSUM_DIGITS - 1; ++j) {
        const int64_t x = acc.digit[j] + carry;
        w[j] = (uint32_t)((uint64_t)x & 0xffffffffu);
        carry = x >> 32;   // floor division by 2^32
    }
    const int64_t top = acc.digit[XSUM_DIGITS - 1] + carry;
    w[XSUM_DIGITS - 1] = (uint32_t)((uint64_t)top & 0xffffffffu);
    w[XSUM_DIGITS] = (uint32_t)((uint64_t)top >> 32);
    w[XSUM_DIGITS + 1] = top < 0 ? 0xffffffffu : 0u;
}

void negate(uint32_t w[kWide])
{
    uint64_t c = 1;
    for (int j = 0; j < kWide; ++j) {
        const uint64_t x = (uint64_t)(uint32_t)~w[j] + c;
        w[j] = (uint32_t)x;
        c = x >> 32;
    }
}

void put32(uint8_t *p, uint32_t v) { std::memcpy(p, &v, 4); }
uint32_t get32(const uint8_t *p)
{
    uint32_t v;
    std::memcpy(&v, p, 4);
    return v;
}

}  // namespace

extern "C" {

xsum_status_t xsum_state_encode(const xsum_acc_t *acc, void *buf, size_t cap, size_t *len)
{
    if (acc == nullptr || len == nullptr)
        return xsum::api_fail(XSUM_EINVAL, "acc or len is NULL");
    for (int j = 0; j < XSUM_DIGITS; ++j)
        if (acc->digit[j] > kDigitLimit || acc->digit[j] < -kDigitLimit)
            return xsum::api_fail(XSUM_ERANGE, "digit " + std::to_string(j) +
                                                   " outside [-2^62, 2^62]");
    if (acc->special > 7u)
        return xsum::api_fail(XSUM_EINVAL, "special bits above bit 2 are set");
    uint32_t w[kWide];
    to_wide(*acc, w);
    const int64_t top = (int64_t)(((uint64_t)w[XSUM_DIGITS] << 32) | w[XSUM_DIGITS - 1]);
    if (top > kTopLimit || top < -kTopLimit)
        return xsum::api_fail(XSUM_ERANGE, "value beyond the encodable range");
    const bool neg = (int32_t)w[kWide - 1] < 0;
    if (neg)
        negate(w);
    int lo = -1, hi = -1;
    for (int j = 0; j < kWide; ++j)
        if (w[j]) {
            if (lo < 0)
                lo = j;
            hi = j;
        }
    const int cnt = lo < 0 ? 0 : hi - lo + 1;
    *len = (size_t)(kHeader + 4 * cnt);
    if (buf == nullptr || cap < *len)
        return xsum::api_fail(XSUM_ERANGE, "buffer too small: " + std::to_string(*len) +
                                               " bytes needed");
    uint8_t *p = (uint8_t *)buf;
    put32(p, kMagic);
    put32(p + 4, acc->special);
    p[8] = (uint8_t)(neg ? 1 : 0);
    p[9] = (uint8_t)(lo < 0 ? 0 : lo);
    p[10] = (uint8_t)cnt;
    p[11] = 0;
    for (int k = 0; k < cnt; ++k)
        put32(p + kHeader + 4 * k, w[lo + k]);
    return XSUM_OK;
}

xsum_status_t xsum_state_decode(const void *buf, size_t len, xsum_acc_t *acc)
{
    if (buf == nullptr || acc == nullptr)
        return xsum::api_fail(XSUM_EINVAL, "buf or acc is NULL");
    const uint8_t *p = (const uint8_t *)buf;
    if (len < (size_t)kHeader || get32(p) != kMagic)
        return xsum::api_fail(XSUM_EINVAL, "not an encoded exact state");
    const uint32_t special = get32(p + 4);
    const int neg = p[8], lo = p[9], cnt = p[10];
    if (special > 7u || neg > 1 || p[11] != 0 || lo + cnt > kWide ||
        len != (size_t)(kHeader + 4 * cnt))
        return xsum::api_fail(XSUM_EINVAL, "malformed encoded exact state");
    uint32_t w[kWide] = {0};
    for (int k = 0; k < cnt; ++k)
        w[lo + k] = get32(p + kHeader + 4 * k);
    if (cnt > 0 && (w[lo] == 0 || w[lo + cnt - 1] == 0))
        return xsum::api_fail(XSUM_EINVAL, "encoded digit run does not start and end non-zero");
    if (neg && cnt == 0)
        return xsum::api_fail(XSUM_EINVAL, "negative zero in an encoded exact state");
    if (w[kWide - 1] != 0 || w[kWide - 2] >= (1u << 30))
        return xsum::api_fail(XSUM_ERANGE, "encoded magnitude beyond the state's range");
    if (neg)
        negate(w);
    const int64_t top =
        (int64_t)(((uint64_t)w[XSUM_DIGITS] << 32) | (uint64_t)w[XSUM_DIGITS - 1]);
    if (top > kTopLimit || top < -kTopLimit)
        return xsum::api_fail(XSUM_ERANGE, "encoded magnitude beyond the state's range");
    std::memset(acc, 0, sizeof(*acc));
    for (int j = 0; j < XSUM_DIGITS - 1; ++j)
        acc->digit[j] = (int64_t)w[j];
    acc->digit[XSUM_DIGITS - 1] = top;
    acc->special = special;
    return XSUM_OK;
}

}  // extern "C"
