// Host-code checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by tests/test_sanitize_cpu.py with g++; no GPU, no HIP runtime):
//   * the exact-state codec (xsum_state_encode / xsum_state_decode) on random
//     valid states and on random and mutated byte strings;
//   * the oracle's exponent-binned C sum on random arrays of all three
//     formats and lengths, where any thread count must give the same bins.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "xsum.h"

namespace xsum {
// the library's error recorder, replaced here (the codec only reports through it)
xsum_status_t api_fail(xsum_status_t st, const std::string &) { return st; }
}  // namespace xsum

extern "C" int oracle_binned_sum(const void *x, uint64_t n, int fmt, int nthreads,
                                 int64_t *out_bins, uint32_t *special);

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAILED %s at line %d\n", #c, __LINE__);             \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

static void codec(std::mt19937_64 &rng)
{
    uint8_t buf[XSUM_STATE_ENCODED_MAX], buf2[XSUM_STATE_ENCODED_MAX];
    for (int it = 0; it < 20000; ++it) {
        xsum_acc_t a;
        std::memset(&a, 0, sizeof(a));
        const int kind = it % 3;
        for (int j = 0; j < XSUM_DIGITS; ++j) {
            int64_t v = (int64_t)(rng() >> 2) - (int64_t(1) << 61);   // |v| <= 2^61
            if (kind == 1 && rng() % 4)
                v = 0;
            if (kind == 2)
                v = (int64_t)(rng() & 0xffffffffu);
            a.digit[j] = v;
        }
        a.digit[XSUM_DIGITS - 1] = (int64_t)(rng() % 7) - 3;
        a.special = (uint32_t)(rng() % 8);
        size_t len = 0;
        CHECK(xsum_state_encode(&a, buf, sizeof(buf), &len) == XSUM_OK);
        CHECK(len >= 12 && len <= XSUM_STATE_ENCODED_MAX && (len - 12) % 4 == 0);
        size_t len2 = 0;
        if (len > 12)
            CHECK(xsum_state_encode(&a, buf2, len - 1, &len2) == XSUM_ERANGE && len2 == len);
        xsum_acc_t b;
        CHECK(xsum_state_decode(buf, len, &b) == XSUM_OK);
        for (int j = 0; j < XSUM_DIGITS - 1; ++j)
            CHECK(b.digit[j] >= 0 && b.digit[j] <= (int64_t)0xffffffffu);
        CHECK(xsum_state_encode(&b, buf2, sizeof(buf2), &len2) == XSUM_OK);
        CHECK(len2 == len && std::memcmp(buf, buf2, len) == 0);
        // mutated and truncated encodings: any status, never a bad access
        for (int m = 0; m < 4; ++m) {
            std::memcpy(buf2, buf, len);
            buf2[rng() % len] ^= (uint8_t)(1u << (rng() % 8));
            const size_t l = (rng() % 3 == 0) ? rng() % (len + 1) : len;
            xsum_acc_t c;
            (void)xsum_state_decode(buf2, l, &c);
        }
    }
    // random byte strings of every length up to the maximum and beyond
    std::vector<uint8_t> junk(400);
    for (int it = 0; it < 20000; ++it) {
        const size_t l = rng() % junk.size();
        for (size_t k = 0; k < l; ++k)
            junk[k] = (uint8_t)rng();
        if (l >= 4 && (it & 1)) {
            const uint32_t magic = 0x31535358u;
            std::memcpy(junk.data(), &magic, 4);
        }
        xsum_acc_t c;
        (void)xsum_state_decode(junk.data(), l, &c);
    }
}

static void oracle_bins(std::mt19937_64 &rng)
{
    std::vector<int64_t> b1(4096), b2(4096);
    for (int it = 0; it < 60; ++it) {
        const int fmt = it % 3;
        const size_t n = (it % 7 == 0) ? 0 : (size_t)(rng() % 300000);
        const size_t es = fmt == 0 ? 8 : fmt == 1 ? 4 : 2;
        std::vector<uint8_t> x(n * es + 1);
        for (auto &v : x)
            v = (uint8_t)rng();
        uint32_t s1 = 0, s2 = 0;
        const int t1 = oracle_binned_sum(n ? x.data() : nullptr, n, fmt, 1, b1.data(), &s1);
        const int t2 = oracle_binned_sum(n ? x.data() : nullptr, n, fmt, 1 + (int)(rng() % 9),
                                         b2.data(), &s2);
        CHECK(t1 == 1 && t2 >= 1);
        CHECK(s1 == s2 && b1 == b2);
    }
    uint32_t s = 0;
    CHECK(oracle_binned_sum(nullptr, 5, 0, 1, b1.data(), &s) == -1);
    CHECK(oracle_binned_sum(b1.data(), 5, 3, 1, b1.data(), &s) == -1);
}

int main()
{
    std::mt19937_64 rng(20161);
    codec(rng);
    oracle_bins(rng);
    std::printf("OK\n");
    return 0;
}
