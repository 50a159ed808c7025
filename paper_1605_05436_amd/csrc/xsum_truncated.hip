// Condition-number-sensitive exact sum for gfx950 (Section 4 of Goodrich &
// Eldawy): one pass sums the input with r-truncated sparse superaccumulators
// and tests the root; the caller squares r and repeats until the test passes.
//
// A sparse superaccumulator here is a list of at most R entries (index i,
// integer value v), most significant first, worth sum v 2^(32 i - 1074).
// Values are exact int64 sums of the radix-2^32 digits added at that index,
// kept without carrying (the one-bit overlap of Section 2 is what makes such
// lazy carries safe: a value is a sum of at most 2^31 digits below 2^32, so it
// stays below 2^63).  An index, once in the list, stays until it is pushed
// out (Section 2: active indices).  Keeping only the top R entries is the
// r-truncation; every dropped part is added, rounded up, to the list's bound
// B = bval 2^(32 bidx - 1074), so the exact sum of everything the list covers
// is within B of its value.
//
// One pass, one launch:
//   1. leaves    each lane walks its share of 16-byte vectors and adds every
//                element's one to three radix-2^32 digits into its list,
//                in order (the lane's share is a path of the summation tree).
//                For r = 2 and 4 the list lives in registers (one compare
//                and select per entry and digit); for r = 16 the same list
//                lives in r LDS slots in index order plus a mask of the
//                active indices, so a digit costs one popcount and one LDS
//                add whatever r is
//   2. tree      lists are merged pairwise up the wave (shuffles), then the
//                block (LDS), then the grid: each block publishes its list in
//                the workspace and the last block to take a ticket merges
//                them (Section 4's bottom-up merge-and-sum, Lemma 3)
//   3. test      the root's value S and bound B: the sum lies in [S-B, S+B];
//                if both ends round (to nearest, ties to even) to the same
//                value v and v is outside the interval, v is the rounded sum
//                and it is inexact.  Otherwise the pass is not certified.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <string>
#include <type_traits>

#include "xsum.h"
#include "xsum_device.h"
#include "xsum_host.h"
#include "xsum_internal.h"

namespace xsum {

xsum_status_t api_fail(xsum_status_t st, const std::string &msg);
xsum_status_t api_hip_fail(hipError_t e, const char *what);
xsum_status_t api_current_cus(int *dev, int *cus);

namespace {

constexpr int kTThreads = 256;
constexpr int kTWaves = kTThreads / 64;
constexpr int kNoIdx = -(1 << 20);
constexpr int kMaxTBlocks = 2048;
constexpr int kTopDigit = 67;       // digit positions of the root's wave layout
constexpr uint64_t kMaxTruncN = 1ull << 31;

// One block's list, published for the last block (256-byte slots).
struct TNode {
    int32_t idx[XSUM_TRUNC_MAX_R];
    int64_t val[XSUM_TRUNC_MAX_R];
    int32_t bidx;
    uint32_t spec;
    uint64_t bval;
};
static_assert(sizeof(TNode) <= 256, "node slot");

struct TCtl {
    uint32_t ticket;
    uint32_t pad[63];
};

// Workspace: control word, node slots, the record of the blocking call, the
// exact-sum state of its untruncated pass.
constexpr size_t kCtlOff = 0;
constexpr size_t kNodesOff = 256;
constexpr size_t kRecOff = kNodesOff + (size_t)kMaxTBlocks * 256;
constexpr size_t kAccOff = kRecOff + 256;
constexpr size_t kWsBytes = kAccOff + ((sizeof(xsum_acc_t) + 255) / 256) * 256;
static_assert(sizeof(xsum_trunc_root_t) <= 256, "record slot");

template <int R>
struct TList {
    int idx[R];
    int64_t val[R];
    int bidx;
    uint64_t bval;
};

__device__ __forceinline__ int64_t add64(int64_t a, int64_t b)
{
    return (int64_t)((uint64_t)a + (uint64_t)b);
}

__device__ __forceinline__ uint64_t mag64(int64_t v)
{
    return v < 0 ? 0ull - (uint64_t)v : (uint64_t)v;
}

__device__ __forceinline__ uint64_t ceil_div_radix(uint64_t v)
{
    return (v >> 32) + ((v & kLow32) != 0);
}

// bound += mag * 2^(32 i), rounded up to the bound's unit.
__device__ __forceinline__ void bound_add(int &bidx, uint64_t &bval, int i, uint64_t mag)
{
    if (mag == 0)
        return;
    if (bval == 0) {
        bidx = i;
        bval = mag;
        return;
    }
    if (i > bidx) {
        bval = (i - bidx >= 2) ? 1ull : ceil_div_radix(bval);
        bidx = i;
    } else if (i < bidx) {
        mag = (bidx - i >= 2) ? 1ull : ceil_div_radix(mag);
    }
    const uint64_t s = bval + mag;
    if (s < bval) {
        // 2^64 + s in units of the next digit, rounded up
        bval = (s >> 32) + (1ull << 32) + 1;
        bidx += 1;
    } else {
        bval = s;
    }
}

template <int R>
__device__ __forceinline__ void tl_clear(TList<R> &L)
{
#pragma unroll
    for (int j = 0; j < R; ++j) {
        L.idx[j] = kNoIdx;
        L.val[j] = 0;
    }
    L.bidx = 0;
    L.bval = 0;
}

// Adds (i, v) for an index i not in the list: below the lowest entry of a
// full list it is dropped; otherwise it takes its place in order and a full
// list drops its lowest entry.
template <int R>
__device__ __forceinline__ void tl_insert(TList<R> &L, int i, int64_t v)
{
    const int lo = L.idx[R - 1];
    const bool full = lo != kNoIdx;
    if (full && i < lo) {
        bound_add(L.bidx, L.bval, i, mag64(v));
        return;
    }
    if (full)
        bound_add(L.bidx, L.bval, lo, mag64(L.val[R - 1]));
    int p = 0;
#pragma unroll
    for (int j = 0; j < R; ++j)
        p += L.idx[j] > i;
#pragma unroll
    for (int j = R - 1; j >= 1; --j) {
        if (j > p) {
            L.idx[j] = L.idx[j - 1];
            L.val[j] = L.val[j - 1];
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j == p) {
            L.idx[j] = i;
            L.val[j] = v;
        }
    }
}

template <int R>
__device__ __forceinline__ void tl_add(TList<R> &L, int i, int64_t v)
{
    bool hit = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (L.idx[j] == i) {
            L.val[j] = add64(L.val[j], v);
            hit = true;
        }
    }
    if (!hit)
        tl_insert(L, i, v);
}

// L += P (Lemma 3: the union of the active indices, values added, then the
// top R kept).
template <int R>
__device__ __forceinline__ void tl_merge(TList<R> &L, const TList<R> &P)
{
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (P.idx[j] != kNoIdx)
            tl_add(L, P.idx[j], P.val[j]);
    bound_add(L.bidx, L.bval, P.bidx, P.bval);
}

__device__ __forceinline__ int64_t shfl_down64(int64_t v, int s)
{
    const uint32_t lo = __shfl_down((uint32_t)v, s, 64);
    const uint32_t hi = __shfl_down((uint32_t)((uint64_t)v >> 32), s, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src)
{
    const uint32_t lo = __shfl((uint32_t)v, src, 64);
    const uint32_t hi = __shfl((uint32_t)((uint64_t)v >> 32), src, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int R>
__device__ __forceinline__ TList<R> tl_shfl_down(const TList<R> &L, int s)
{
    TList<R> P;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        P.idx[j] = __shfl_down(L.idx[j], s, 64);
        P.val[j] = shfl_down64(L.val[j], s);
    }
    P.bidx = __shfl_down(L.bidx, s, 64);
    P.bval = (uint64_t)shfl_down64((int64_t)L.bval, s);
    return P;
}

// Lane 0 ends with the merge of the wave's lists.
template <int R>
__device__ __forceinline__ void tl_wave_merge(TList<R> &L, int lane, int width)
{
#pragma unroll 1
    for (int s = width >> 1; s >= 1; s >>= 1) {
        const TList<R> P = tl_shfl_down(L, s);
        if (lane < s)
            tl_merge(L, P);
    }
}

// A lane's list while it walks its elements.  To keep the per-entry update
// to one select chain and one 64-bit add, a negative element adds the
// complement ~d (= -d - 1) of its digit to the entries it touches and -1 to
// every other entry; `negs` counts negative elements and base[j] is `negs`
// when entry j was created, so the entry's true value is
// val[j] + (negs - base[j]).  Elements dropped whole below the lowest entry
// of a full list (each below one unit of that entry) are counted in `drops`
// and moved into the bound whenever the lowest entry may change.
template <int R>
struct TWalk {
    TList<R> L;
    uint32_t base[R];
    uint32_t negs;
    uint32_t drops;
    uint32_t spec;
    uint32_t emax;
};

template <int R>
__device__ __forceinline__ void tw_init(TWalk<R> &W)
{
    tl_clear(W.L);
#pragma unroll
    for (int j = 0; j < R; ++j)
        W.base[j] = 0;
    W.negs = 0;
    W.drops = 0;
    W.spec = 0;
    W.emax = 0;
}

template <int R>
__device__ __forceinline__ void tw_flush_drops(TWalk<R> &W)
{
    if (W.drops) {
        bound_add(W.L.bidx, W.L.bval, W.L.idx[R - 1], W.drops);
        W.drops = 0;
    }
}

// tl_insert on the biased list: the entry pushed out is bounded by its true
// value, and the new entry (exact value v) starts unbiased.
template <int R>
__device__ __forceinline__ void tw_insert(TWalk<R> &W, int i, int64_t v)
{
    TList<R> &L = W.L;
    const int lo = L.idx[R - 1];
    const bool full = lo != kNoIdx;
    if (full && i < lo) {
        bound_add(L.bidx, L.bval, i, mag64(v));
        return;
    }
    if (full)
        bound_add(L.bidx, L.bval, lo,
                  mag64(add64(L.val[R - 1], (int64_t)(W.negs - W.base[R - 1]))));
    int p = 0;
#pragma unroll
    for (int j = 0; j < R; ++j)
        p += L.idx[j] > i;
#pragma unroll
    for (int j = R - 1; j >= 1; --j) {
        if (j > p) {
            L.idx[j] = L.idx[j - 1];
            L.val[j] = L.val[j - 1];
            W.base[j] = W.base[j - 1];
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j == p) {
            L.idx[j] = i;
            L.val[j] = v;
            W.base[j] = W.negs;
        }
    }
}

// The walk's list as a plain list (true values, drops in the bound).
template <int R>
__device__ __forceinline__ void tw_finish(TWalk<R> &W)
{
    tw_flush_drops(W);
#pragma unroll
    for (int j = 0; j < R; ++j)
        W.L.val[j] = W.L.idx[j] != kNoIdx
                         ? add64(W.L.val[j], (int64_t)(W.negs - W.base[j]))
                         : 0;
}

// One element given as its sign and radix-2^32 digits d0, d1, d2 at indices
// k, k+1, k+2 (ND of them may be non-zero).  Digits whose index is in the
// list are added in place.  The others are dropped together when all lie
// below the lowest entry of a full list (their sum is below one unit of that
// entry); otherwise each is inserted.
template <int R, int ND>
__device__ __forceinline__ void tw_add_leaf(TWalk<R> &W, int k, uint32_t d0,
                                            uint32_t d1, uint32_t d2, bool neg)
{
    const uint32_t sm = neg ? ~0u : 0u;
    const uint32_t x0 = d0 ^ sm, x1 = d1 ^ sm, x2 = d2 ^ sm;
    const int k1 = k + 1, k2 = k + 2;
    W.negs -= sm;  // sm is all ones for a negative element: this adds one
    bool h0 = false, h1 = false, h2 = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int ij = W.L.idx[j];
        const bool e0 = ij == k, e1 = ij == k1, e2 = ND == 3 && ij == k2;
        const uint32_t lo = e0 ? x0 : (e1 ? x1 : (e2 ? x2 : sm));
        // val += (sm << 32) | lo as two 32-bit adds (one carry)
        uint32_t c;
        const uint32_t vlo = __builtin_addc((uint32_t)W.L.val[j], lo, 0u, &c);
        const uint32_t vhi = (uint32_t)((uint64_t)W.L.val[j] >> 32) + sm + c;
        W.L.val[j] = (int64_t)(((uint64_t)vhi << 32) | vlo);
        h0 |= e0;
        h1 |= e1;
        h2 |= e2;
    }
    const bool m0 = d0 != 0 && !h0;
    const bool m1 = d1 != 0 && !h1;
    const bool m2 = ND == 3 && d2 != 0 && !h2;
    // the common miss (everything missing lies below a full list) is counted
    // without a branch; only insertions branch
    const bool miss = m0 || m1 || m2;
    const int lo = W.L.idx[R - 1];
    const int top = m2 ? k2 : (m1 ? k1 : k);
    const bool drop = lo != kNoIdx && top < lo;
    W.drops += (miss && drop) ? 1u : 0u;
    if (miss && !drop) {
        tw_flush_drops(W);
        if (m2)
            tw_insert(W, k2, neg ? -(int64_t)d2 : (int64_t)d2);
        if (m1)
            tw_insert(W, k1, neg ? -(int64_t)d1 : (int64_t)d1);
        if (m0)
            tw_insert(W, k, neg ? -(int64_t)d0 : (int64_t)d0);
    }
}

template <int R>
struct RegWalk : TWalk<R> {
    template <int ND>
    __device__ __forceinline__ void add_leaf(int k, uint32_t d0, uint32_t d1, uint32_t d2, bool neg)
    {
        tw_add_leaf<R, ND>(*this, k, d0, d1, d2, neg);
    }
    __device__ __forceinline__ void finish(TList<R> &out)
    {
        tw_finish(*this);
        out = this->L;
    }
};

// +d or -d (m = 0 or all ones) as a 64-bit two's complement value: the low
// word (d ^ m) - m, the high word m - m minus the borrow.
__device__ __forceinline__ int64_t signed_digit(uint32_t d, uint32_t m)
{
    uint32_t b;
    const uint32_t lo = __builtin_subc(d ^ m, m, 0u, &b);
    const uint32_t hi = __builtin_subc(m, m, b, &b);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A lane's list kept in LDS as R slots in decreasing index order (slot j at
// col[j * kTThreads]) plus a mask of the active indices in registers: the
// slot of an active index is the number of active indices above it, so a
// digit whose index is active costs one popcount and one LDS add whatever r
// is, and the list takes R * 8 bytes per lane (several waves per SIMD).
// Slots at or past the entry count hold stale values and are never read.
template <int R>
struct SlotWalk {
    uint64_t *col;
    uint64_t act;     // active indices 0..63
    uint32_t acth;    // active indices 64, 65
    int cnt;          // active indices
    int lo;           // the lowest active index when cnt == R, else kNoIdx
    int bidx;
    uint64_t bval;
    uint32_t drops, spec, emax;

    __device__ __forceinline__ void init(uint64_t *c)
    {
        col = c;
        act = 0;
        acth = 0;
        cnt = 0;
        lo = kNoIdx;
        bidx = 0;
        bval = 0;
        drops = 0;
        spec = 0;
        emax = 0;
    }
    __device__ __forceinline__ void set_bit(int i)
    {
        if (i < 64)
            act |= 1ull << i;
        else
            acth |= 1u << (i - 64);
    }
    __device__ __forceinline__ void clear_bit(int i)
    {
        if (i < 64)
            act &= ~(1ull << i);
        else
            acth &= ~(1u << (i - 64));
    }
    __device__ __forceinline__ int lowest() const
    {
        return act ? __builtin_ctzll(act) : 64 + __builtin_ctz(acth);
    }
    __device__ __forceinline__ int highest() const
    {
        return acth ? 95 - __builtin_clz(acth) : (act ? 63 - __builtin_clzll(act) : kNoIdx);
    }
    // number of active indices above i (0 <= i <= 65)
    __device__ __forceinline__ int above(int i) const
    {
        const int s = i + 1;
        const uint32_t h = s >= 64 ? acth >> (s - 64) : acth;
        const uint64_t l = s < 64 ? act >> s : 0ull;
        return __builtin_popcount(h) + __builtin_popcountll(l);
    }
    // the mask from index k up (k <= 63): bit b is index k + b, the two
    // indices above 63 shifted in below the top
    __device__ __forceinline__ uint64_t window(int k) const
    {
        return (act >> k) | (((uint64_t)acth << 1) << (63 - k));
    }
    __device__ __forceinline__ uint64_t *slot(int j) const { return col + j * kTThreads; }
    __device__ __forceinline__ void flush()
    {
        if (drops) {
            bound_add(bidx, bval, lo, drops);
            drops = 0;
        }
    }
    // (i, v) for an inactive index i
    __device__ __forceinline__ void insert(int i, int64_t v)
    {
        if (i < lo) {
            bound_add(bidx, bval, i, mag64(v));
            return;
        }
        if (cnt == R) {
            // the lowest entry is the last slot
            const int64_t ev = (int64_t)lds_load(slot(R - 1));
            clear_bit(lo);
            --cnt;
            bound_add(bidx, bval, lo, mag64(ev));
            lo = kNoIdx;
        }
        // the entries below i move down one slot
        const int p = above(i);
#pragma unroll 1
        for (int j = cnt - 1; j >= p; --j)
            lds_store(slot(j + 1), lds_load(slot(j)));
        lds_store(slot(p), (uint64_t)v);
        set_bit(i);
        ++cnt;
        if (cnt == R)
            lo = lowest();
    }
    template <int ND>
    __device__ __forceinline__ void add_leaf(int k, uint32_t d0, uint32_t d1, uint32_t d2, bool neg)
    {
        // which of the indices k..k+2 (k <= 63) are active
        const uint64_t wdw = window(k);
        const uint32_t on = (uint32_t)wdw & 7u;
        const uint32_t nz = (d0 != 0 ? 1u : 0u) | (d1 != 0 ? 2u : 0u) |
                            (ND == 3 && d2 != 0 ? 4u : 0u);
        const uint32_t sm = neg ? ~0u : 0u;
        const int64_t s0 = signed_digit(d0, sm);
        const int64_t s1 = signed_digit(d1, sm);
        const int64_t s2 = ND == 3 ? signed_digit(d2, sm) : 0;
        const uint32_t hit = nz & on;
        // slots of k+2, k+1, k: the active indices above k+2 are the window's
        // bits from 3 up and, for k < 2, the indices above 63 past its top;
        // each index's slot is one past the one above it when that is active
        const int a2 = __builtin_popcountll(wdw >> 3) +
                       __builtin_popcount((uint32_t)((uint64_t)acth >> k));
        const int a1 = a2 + (int)((on >> 2) & 1u);
        const int a0 = a1 + (int)((on >> 1) & 1u);
        if (hit & 1u)
            lds_add(slot(a0), (uint64_t)s0);
        if (hit & 2u)
            lds_add(slot(a1), (uint64_t)s1);
        if (ND == 3 && (hit & 4u))
            lds_add(slot(a2), (uint64_t)s2);
        const uint32_t miss = nz & ~on;
        const int top = k + 31 - __builtin_clz(miss | 1u);
        const bool drop = top < lo;     // below a full list
        drops += (miss && drop) ? 1u : 0u;
        if (miss && !drop) {
            flush();
#pragma unroll 1
            for (int c = 2; c >= 0; --c)
                if ((miss >> c) & 1u)
                    insert(k + c, c == 2 ? s2 : (c == 1 ? s1 : s0));
        }
    }
    __device__ __forceinline__ void finish(TList<R> &out)
    {
        flush();
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int h = highest();
            if (h != kNoIdx) {
                out.idx[j] = h;
                out.val[j] = (int64_t)lds_load(slot(j));
                clear_bit(h);
            } else {
                out.idx[j] = kNoIdx;
                out.val[j] = 0;
            }
        }
        out.bidx = bidx;
        out.bval = bval;
    }
};

// Element decoders: exponent position q of the significand's bit 0 in units
// of 2^-1074, split at the radix-2^32 digit boundary.  Infinities and NaNs
// add nothing; the walk keeps the largest exponent field it met (emax), and
// the tile loop records the special values of a tile where it is all ones.
template <typename WT>
__device__ __forceinline__ void leaf_f64(WT &W, uint32_t lo, uint32_t hi)
{
    const uint32_t e = (hi >> 20) & 0x7ffu;
    W.emax = max(W.emax, e);
    const bool neg = (hi >> 31) != 0;
    const bool special = e == 0x7ffu;
    const uint32_t mh = special ? 0u : ((hi & 0xfffffu) | (e ? 0x100000u : 0u));
    const uint64_t m = ((uint64_t)mh << 32) | (special ? 0u : lo);
    const int q = e ? (int)e - 1 : 0;
    const int s = q & 31;
    const uint64_t w = m << s;
    const uint32_t d2 = s ? (uint32_t)(m >> (64 - s)) : 0u;
    W.template add_leaf<3>(q >> 5, (uint32_t)w, (uint32_t)(w >> 32), d2, neg);
}

template <typename WT>
__device__ __forceinline__ void leaf_f32(WT &W, uint32_t b)
{
    const uint32_t e = (b >> 23) & 0xffu;
    W.emax = max(W.emax, e);
    const bool neg = (b >> 31) != 0;
    const uint32_t m = e == 0xffu ? 0u : ((b & 0x7fffffu) | (e ? 1u << 23 : 0u));
    const int q = (e ? (int)e - 1 : 0) + 925;
    const uint64_t w = (uint64_t)m << (q & 31);
    W.template add_leaf<2>(q >> 5, (uint32_t)w, (uint32_t)(w >> 32), 0u, neg);
}

template <typename WT>
__device__ __forceinline__ void leaf_bf16(WT &W, uint32_t h)
{
    const uint32_t e = (h >> 7) & 0xffu;
    W.emax = max(W.emax, e);
    const bool neg = ((h >> 15) & 1u) != 0;
    const uint32_t m = e == 0xffu ? 0u : ((h & 0x7fu) | (e ? 1u << 7 : 0u));
    const int q = (e ? (int)e - 1 : 0) + 941;
    const uint64_t w = (uint64_t)m << (q & 31);
    W.template add_leaf<2>(q >> 5, (uint32_t)w, (uint32_t)(w >> 32), 0u, neg);
}

// Special-value bits of one element (0 for a finite one).
__device__ __forceinline__ uint32_t spec_f64(uint32_t lo, uint32_t hi)
{
    return ((hi >> 20) & 0x7ffu) == 0x7ffu
               ? special_bits(((hi & 0xfffffu) | lo) != 0, (hi >> 31) != 0)
               : 0u;
}

__device__ __forceinline__ uint32_t spec_f32(uint32_t b)
{
    return ((b >> 23) & 0xffu) == 0xffu ? special_bits((b & 0x7fffffu) != 0, (b >> 31) != 0)
                                        : 0u;
}

__device__ __forceinline__ uint32_t spec_bf16(uint32_t h)
{
    return ((h >> 7) & 0xffu) == 0xffu ? special_bits((h & 0x7fu) != 0, ((h >> 15) & 1u) != 0)
                                       : 0u;
}

template <int FMT>
__device__ __forceinline__ uint32_t spec_vector(const vec4u &q)
{
    if constexpr (FMT == XSUM_F64) {
        return spec_f64(q.x, q.y) | spec_f64(q.z, q.w);
    } else if constexpr (FMT == XSUM_F32) {
        return spec_f32(q.x) | spec_f32(q.y) | spec_f32(q.z) | spec_f32(q.w);
    } else {
        uint32_t r = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            r |= spec_bf16(q[c] & 0xffffu) | spec_bf16(q[c] >> 16);
        return r;
    }
}

// the exponent field of an infinity or NaN
template <int FMT>
constexpr uint32_t kAllOnes = FMT == XSUM_F64 ? 0x7ffu : 0xffu;

template <int FMT, typename WT>
__device__ __forceinline__ void add_vector(WT &W, const vec4u &q)
{
    if constexpr (FMT == XSUM_F64) {
        leaf_f64(W, q.x, q.y);
        leaf_f64(W, q.z, q.w);
    } else if constexpr (FMT == XSUM_F32) {
        leaf_f32(W, q.x);
        leaf_f32(W, q.y);
        leaf_f32(W, q.z);
        leaf_f32(W, q.w);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            leaf_bf16(W, q[c] & 0xffffu);
            leaf_bf16(W, q[c] >> 16);
        }
    }
}

template <int FMT, typename WT>
__device__ __forceinline__ void add_one(WT &W, const uint8_t *p)
{
    if constexpr (FMT == XSUM_F64) {
        const uint32_t *w = (const uint32_t *)p;
        leaf_f64(W, w[0], w[1]);
        W.spec |= spec_f64(w[0], w[1]);
    } else if constexpr (FMT == XSUM_F32) {
        const uint32_t b = *(const uint32_t *)p;
        leaf_f32(W, b);
        W.spec |= spec_f32(b);
    } else {
        const uint32_t h = *(const uint16_t *)p;
        leaf_bf16(W, h);
        W.spec |= spec_bf16(h);
    }
}

template <typename T>
__device__ __forceinline__ void sys_store(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__device__ __forceinline__ T sys_load(T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Adds the value v at digit position i to the wave's digit layout (lane l
// holds digits 2l in a and 2l+1 in b).
__device__ __forceinline__ void put_digit(int64_t &a, int64_t &b, int lane, int i, int64_t v)
{
    a += i == 2 * lane ? v : 0;
    b += i == 2 * lane + 1 ? v : 0;
}

// Sign of the normalised wave value: -1, 0 or +1.
__device__ __forceinline__ int wave_sign(int64_t a, int64_t b)
{
    const int64_t top = __shfl(b, 33, 64);
    if (top < 0)
        return -1;
    return __ballot(a != 0 || b != 0) ? 1 : 0;
}

// value of a finite result bit pattern in out_fmt, as digits: k, (d0, d1, d2)
__device__ __forceinline__ void result_digits(uint64_t bits, int out_fmt, bool &neg, int &k,
                                              uint32_t &d0, uint32_t &d1, uint32_t &d2)
{
    uint64_t m;
    int q;
    if (out_fmt == XSUM_F64) {
        const uint32_t e = (uint32_t)(bits >> 52) & 0x7ffu;
        neg = (bits >> 63) != 0;
        m = (bits & ((1ull << 52) - 1)) | (e ? 1ull << 52 : 0ull);
        q = e ? (int)e - 1 : 0;
    } else if (out_fmt == XSUM_F32) {
        const uint32_t e = (uint32_t)(bits >> 23) & 0xffu;
        neg = ((bits >> 31) & 1u) != 0;
        m = (bits & 0x7fffffu) | (e ? 1u << 23 : 0u);
        q = (e ? (int)e - 1 : 0) + 925;
    } else {
        const uint32_t e = (uint32_t)(bits >> 7) & 0xffu;
        neg = ((bits >> 15) & 1u) != 0;
        m = (bits & 0x7fu) | (e ? 1u << 7 : 0u);
        q = (e ? (int)e - 1 : 0) + 941;
    }
    const int s = q & 31;
    const uint64_t w = m << s;
    k = q >> 5;
    d0 = (uint32_t)w;
    d1 = (uint32_t)(w >> 32);
    d2 = s ? (uint32_t)(m >> (64 - s)) : 0u;
}

__device__ __forceinline__ bool is_inf_or_nan(uint64_t bits, int out_fmt)
{
    const OutFormat f = out_format(out_fmt);
    return ((bits >> f.t) & f.emax) == f.emax;
}

// The stopping test on the root list held by lane 0, run by one full wave.
// Writes the record (root entries, bound, result) with plain stores from
// lane 0.
template <int R>
__device__ __forceinline__ void finish_root(const TList<R> &L, uint32_t spec, int r, int out_fmt,
                            xsum_trunc_root_t *rec, int lane)
{
    int64_t a = 0, b = 0;
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = __shfl(L.idx[j], 0, 64);
        const int64_t v = shfl64(L.val[j], 0);
        if (i != kNoIdx) {
            ++cnt;
            put_digit(a, b, lane, i, (int64_t)((uint64_t)v & kLow32));
            put_digit(a, b, lane, i + 1, v >> 32);
        }
    }
    const int bidx = __shfl(L.bidx, 0, 64);
    const uint64_t bval = (uint64_t)shfl64((int64_t)L.bval, 0);
    const OutFormat f = out_format(out_fmt);
    uint32_t flags = 0;
    uint64_t bits = 0;
    bool ok;
    if (special_result(spec, f, bits, flags)) {
        ok = true;
    } else if (bval == 0) {
        normalise_wave(a, b, lane);
        bits = round_wave(a, b, lane, 0, out_fmt, flags);
        ok = true;
    } else if (bidx + 1 > kTopDigit) {
        ok = false;
    } else {
        const int64_t blo = (int64_t)(bval & kLow32), bhi = (int64_t)(bval >> 32);
        int64_t la = a, lb = b, ha = a, hb = b;
        put_digit(la, lb, lane, bidx, -blo);
        put_digit(la, lb, lane, bidx + 1, -bhi);
        put_digit(ha, hb, lane, bidx, blo);
        put_digit(ha, hb, lane, bidx + 1, bhi);
        normalise_wave(la, lb, lane);
        normalise_wave(ha, hb, lane);
        uint32_t fl, fh;
        const uint64_t bl = round_wave(la, lb, lane, 0, out_fmt, fl);
        const uint64_t bh = round_wave(ha, hb, lane, 0, out_fmt, fh);
        ok = bl == bh;
        if (ok && !is_inf_or_nan(bl, out_fmt)) {
            // the rounded value must lie outside [S - B, S + B]
            bool neg;
            int k;
            uint32_t d0, d1, d2;
            result_digits(bl, out_fmt, neg, k, d0, d1, d2);
            const int64_t sg = neg ? 1 : -1;  // adds -value
            put_digit(la, lb, lane, k, sg * (int64_t)d0);
            put_digit(la, lb, lane, k + 1, sg * (int64_t)d1);
            put_digit(la, lb, lane, k + 2, sg * (int64_t)d2);
            put_digit(ha, hb, lane, k, sg * (int64_t)d0);
            put_digit(ha, hb, lane, k + 1, sg * (int64_t)d1);
            put_digit(ha, hb, lane, k + 2, sg * (int64_t)d2);
            normalise_wave(la, lb, lane);
            normalise_wave(ha, hb, lane);
            const int sl = wave_sign(la, lb), sh = wave_sign(ha, hb);
            ok = sl == sh && sl != 0;
        }
        bits = bl;
        flags = fl | fh;
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            rec->index[j] = L.idx[j];
            rec->value[j] = L.val[j];
        }
#pragma unroll
        for (int j = R; j < XSUM_TRUNC_MAX_R; ++j) {
            rec->index[j] = kNoIdx;
            rec->value[j] = 0;
        }
        rec->count = (uint32_t)cnt;
        rec->bound_index = bidx;
        rec->bound_value = bval;
        rec->special = spec;
        rec->certified = ok ? 1u : 0u;
        rec->bits = ok ? bits : 0ull;
        rec->flags = ok ? flags : 0u;
        rec->r = (uint32_t)r;
    }
}

template <int FMT, int R, int U, bool COL>
__global__ __launch_bounds__(kTThreads) void truncated_kernel(
    const uint8_t *__restrict__ x, uint32_t head, uint64_t nvec, uint32_t tail,
    TCtl *ctl, TNode *nodes, xsum_trunc_root_t *rec, int out_fmt)
{
    using G = Geo<FMT>;
    __shared__ TList<R> wl[kTWaves];
    __shared__ uint32_t blk_spec;
    __shared__ int is_last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0)
        blk_spec = 0;
    __shared__ uint64_t cols[COL ? R : 1][kTThreads];
    std::conditional_t<COL, SlotWalk<R>, RegWalk<R>> W;
    if constexpr (COL)
        W.init(&cols[0][tid]);
    else
        tw_init(W);

    // 1. leaves: vectors tid + j*T of each tile of U*T (T threads in the grid)
    const vec4u *v = (const vec4u *)(x + (uint64_t)head * G::kBytes);
    const uint64_t T = (uint64_t)gridDim.x * kTThreads;
    for (uint64_t tb = (uint64_t)blockIdx.x * kTThreads; tb < nvec; tb += U * T) {
        const uint64_t base = tb + tid;
        vec4u q[U];
        if (tb + (kTThreads - 1) + (uint64_t)(U - 1) * T < nvec) {
            // the whole block's tile is in range
#pragma unroll
            for (int j = 0; j < U; ++j)
                q[j] = __builtin_nontemporal_load(v + base + (uint64_t)j * T);
        } else {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const uint64_t i = base + (uint64_t)j * T;
                q[j] = vec4u{0u, 0u, 0u, 0u};
                if (i < nvec)
                    q[j] = __builtin_nontemporal_load(v + i);
            }
        }
#pragma clang loop unroll(full)
        for (int j = 0; j < U; ++j)
            add_vector<FMT>(W, q[j]);
        if (__builtin_expect(W.emax == kAllOnes<FMT>, 0)) {
            // rare: read the tile again rather than keep it in registers
#pragma unroll 1
            for (int j = 0; j < U; ++j) {
                const uint64_t i = base + (uint64_t)j * T;
                if (i < nvec)
                    W.spec |= spec_vector<FMT>(v[i]);
            }
        }
        W.emax = 0;
    }
    if (blockIdx.x == 0) {
        if ((uint32_t)tid < head)
            add_one<FMT>(W, x + (uint64_t)tid * G::kBytes);
        if ((uint32_t)tid < tail)
            add_one<FMT>(W, x + (uint64_t)head * G::kBytes + nvec * 16 +
                                (uint64_t)tid * G::kBytes);
    }
    TList<R> L;
    W.finish(L);
    const uint32_t spec = W.spec;

    // 2. tree: wave, block, grid
    tl_wave_merge(L, lane, 64);
    __syncthreads();  // blk_spec is zero
    if (spec)
        atomicOr(&blk_spec, spec);
    if (lane == 0)
        wl[wave] = L;
    __syncthreads();
    if (wave == 0) {
        if (lane < kTWaves)
            L = wl[lane];
        else
            tl_clear(L);
        tl_wave_merge(L, lane, kTWaves);
        if (lane == 0) {
            TNode *nd = nodes + blockIdx.x;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                sys_store(&nd->idx[j], L.idx[j]);
                sys_store(&nd->val[j], L.val[j]);
            }
            sys_store(&nd->bidx, L.bidx);
            sys_store(&nd->bval, L.bval);
            sys_store(&nd->spec, blk_spec);
        }
    }
    // the node's stores have completed at the memory side before the ticket
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
        const unsigned t = __hip_atomic_fetch_add(&ctl->ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last || wave != 0)
        return;

    // the last block: lane l merges nodes l, l+64, ... in order, then the wave
    tl_clear(L);
    uint32_t gspec = 0;
    for (uint32_t bk = lane; bk < gridDim.x; bk += 64) {
        TNode *nd = nodes + bk;
        TList<R> P;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            P.idx[j] = sys_load(&nd->idx[j]);
            P.val[j] = sys_load(&nd->val[j]);
        }
        P.bidx = sys_load(&nd->bidx);
        P.bval = sys_load(&nd->bval);
        gspec |= sys_load(&nd->spec);
        tl_merge(L, P);
    }
    tl_wave_merge(L, lane, 64);
#pragma unroll
    for (int bit = 1; bit <= 4; bit <<= 1)
        if (__ballot((gspec & bit) != 0))
            gspec |= bit;

    // 3. test
    finish_root(L, gspec, R, out_fmt, rec, lane);
    if (lane == 0)
        sys_store(&ctl->ticket, 0u);
}

template <int FMT, int R>
hipError_t launch_round_fmt(const void *x, uint64_t n, TCtl *ctl, TNode *nodes,
                            xsum_trunc_root_t *rec, int out_fmt, int cus, hipStream_t s)
{
    // r = 16: the LDS slots (one add per digit whatever r is); r = 2 and
    // 4: the register list (fewer entries to compare)
    constexpr bool COL = R > 4;
    constexpr int U = 8;
    using G = Geo<FMT>;
    const uintptr_t addr = (uintptr_t)x;
    uint64_t head = addr % 16 ? (16 - addr % 16) / G::kBytes : 0;
    if (head > n)
        head = n;
    const uint64_t body = (n - head) * G::kBytes;
    const uint64_t nvec = body / 16;
    const uint32_t tail = (uint32_t)((body % 16) / G::kBytes);
    const uint64_t per_block = (uint64_t)kTThreads * U;
    uint64_t blocks = (nvec + per_block - 1) / per_block;
    // one resident wave of blocks: as many per compute unit as registers
    // and LDS allow (a block past that would run alone at the end); asked
    // once per instance, on the first call's device (the answer depends only
    // on the kernel and the architecture)
    static const int per_cu = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, truncated_kernel<FMT, R, U, COL>, kTThreads, 0) != hipSuccess || nb < 1)
            nb = 1;
        return nb;
    }();
    const uint64_t cap = (uint64_t)cus * (uint64_t)per_cu;
    if (blocks > cap)
        blocks = cap;
    if (blocks > (uint64_t)kMaxTBlocks)
        blocks = kMaxTBlocks;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL((truncated_kernel<FMT, R, U, COL>), dim3((unsigned)blocks), dim3(kTThreads),
                       0, s, (const uint8_t *)x, (uint32_t)head, nvec, tail, ctl, nodes, rec,
                       out_fmt);
    return hipGetLastError();
}

template <int FMT>
hipError_t launch_round_r(const void *x, uint64_t n, int r, TCtl *ctl, TNode *nodes,
                          xsum_trunc_root_t *rec, int out_fmt, int cus, hipStream_t s)
{
    if (r == 2)
        return launch_round_fmt<FMT, 2>(x, n, ctl, nodes, rec, out_fmt, cus, s);
    if (r == 4)
        return launch_round_fmt<FMT, 4>(x, n, ctl, nodes, rec, out_fmt, cus, s);
    return launch_round_fmt<FMT, 16>(x, n, ctl, nodes, rec, out_fmt, cus, s);
}

hipError_t launch_round(const void *x, uint64_t n, int dtype, int r, void *ws,
                        xsum_trunc_root_t *rec, int out_fmt, int cus, hipStream_t s)
{
    TCtl *ctl = (TCtl *)((uint8_t *)ws + kCtlOff);
    TNode *nodes = (TNode *)((uint8_t *)ws + kNodesOff);
    if (dtype == XSUM_F64)
        return launch_round_r<XSUM_F64>(x, n, r, ctl, nodes, rec, out_fmt, cus, s);
    if (dtype == XSUM_F32)
        return launch_round_r<XSUM_F32>(x, n, r, ctl, nodes, rec, out_fmt, cus, s);
    return launch_round_r<XSUM_BF16>(x, n, r, ctl, nodes, rec, out_fmt, cus, s);
}

bool valid_fmt(int f) { return f == XSUM_F64 || f == XSUM_F32 || f == XSUM_BF16; }

xsum_status_t check_args(const void *x, uint64_t n, int dtype, int out_dtype, void *ws,
                         size_t ws_bytes, int *of)
{
    if (!valid_fmt(dtype))
        return api_fail(XSUM_EDTYPE, "unknown input dtype " + std::to_string(dtype));
    *of = resolve_out(dtype, out_dtype);
    if (!valid_fmt(*of))
        return api_fail(XSUM_EDTYPE, "unknown output dtype " + std::to_string(out_dtype));
    if (n > 0 && x == nullptr)
        return api_fail(XSUM_EINVAL, "x is NULL with n > 0");
    if ((uintptr_t)x % element_size(dtype))
        return api_fail(XSUM_EINVAL, "x is not aligned to its element size");
    if (n > kMaxTruncN)
        return api_fail(XSUM_ERANGE, "the truncated pass takes at most 2^31 elements");
    if (ws == nullptr || (uintptr_t)ws % 256)
        return api_fail(XSUM_EINVAL, "workspace is NULL or not 256-byte aligned");
    if (ws_bytes < kWsBytes)
        return api_fail(XSUM_EINVAL, "workspace smaller than xsum_truncated_workspace_size()");
    return XSUM_OK;
}

}  // namespace
}  // namespace xsum

extern "C" {

size_t xsum_truncated_workspace_size(void) { return xsum::kWsBytes; }

xsum_status_t xsum_truncated_round(const void *x, uint64_t n, int dtype, int out_dtype,
                                   int r, xsum_trunc_root_t *root_dev, void *workspace,
                                   size_t ws_bytes, void *stream)
{
    int of;
    xsum_status_t st = xsum::check_args(x, n, dtype, out_dtype, workspace, ws_bytes, &of);
    if (st != XSUM_OK)
        return st;
    if (r != 2 && r != 4 && r != 16)
        return xsum::api_fail(XSUM_EINVAL, "r must be 2, 4 or 16");
    if (root_dev == nullptr)
        return xsum::api_fail(XSUM_EINVAL, "root_dev is NULL");
    int dev, cus;
    if ((st = xsum::api_current_cus(&dev, &cus)) != XSUM_OK)
        return st;
    hipError_t e = xsum::launch_round(x, n, dtype, r, workspace, root_dev, of, cus,
                                      (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : xsum::api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_exact_sum_truncated(const void *x, uint64_t n, int dtype, int out_dtype,
                                       void *out_host, uint32_t *flags_host, int *r_host,
                                       void *workspace, size_t ws_bytes, void *stream)
{
    int of;
    xsum_status_t st = xsum::check_args(x, n, dtype, out_dtype, workspace, ws_bytes, &of);
    if (st != XSUM_OK)
        return st;
    if (out_host == nullptr)
        return xsum::api_fail(XSUM_EINVAL, "out_host is NULL");
    int dev, cus;
    if ((st = xsum::api_current_cus(&dev, &cus)) != XSUM_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    xsum_trunc_root_t *rec = (xsum_trunc_root_t *)(ws + xsum::kRecOff);
    xsum_acc_t *acc = (xsum_acc_t *)(ws + xsum::kAccOff);
    hipError_t e = xsum::launch_zero_words((uint64_t *)ws, xsum::kWsBytes / 8, s);
    if (e != hipSuccess)
        return xsum::api_hip_fail(e, "workspace fill");
    xsum_trunc_root_t h;
    int r = 2;
    for (; r <= 16; r *= r) {
        e = xsum::launch_round(x, n, dtype, r, ws, rec, of, cus, s);
        if (e != hipSuccess)
            return xsum::api_hip_fail(e, "kernel launch");
        e = hipMemcpyAsync(&h, rec, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return xsum::api_hip_fail(e, "record copy");
        if (h.certified)
            break;
    }
    if (r > 16) {
        // r = 256 exceeds the number of digit positions: nothing would be
        // truncated, so this pass is the exact sum itself
        xsum::Finish fin{xsum::kRound, of, &rec->bits, &rec->flags, 1};
        e = xsum::launch_accumulate(x, n, dtype, acc, fin, cus, xsum::Shape{0}, s);
        if (e != hipSuccess)
            return xsum::api_hip_fail(e, "kernel launch");
        e = hipMemcpyAsync(&h, rec, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return xsum::api_hip_fail(e, "record copy");
        r = 0;
    }
    const int nb = xsum::out_bytes(of);
    memcpy(out_host, &h.bits, nb);
    if (flags_host)
        *flags_host = h.flags;
    if (r_host)
        *r_host = r;
    return XSUM_OK;
}

}  // extern "C"
