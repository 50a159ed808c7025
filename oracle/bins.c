/*
 * Exponent-binned exact accumulation of IEEE binary floats, for the oracle.
 *
 * TEST INFRASTRUCTURE ONLY: called from the oracle's Python wrapper, never by
 * the product library, and shares no code with it.
 *
 * The exact sum of the inputs is the wide fixed-point integer of Section 2 of
 * the paper.  Instead of shifting each significand into place, inputs with the
 * same biased exponent E have the same scale, so this routine adds the signed
 * integer significands of all inputs with exponent E into one 128-bit bin:
 *
 *     bin[E] += (-1)^s * m,   m = M + (E != 0) * 2^t
 *
 * A significand is below 2^53, so a 128-bit bin absorbs 2^74 additions
 * without overflow.  The caller then forms sum_E bin[E] * 2^(max(E,1) - 1 -
 * bias - t), a big integer, exactly.  Threads split the input into contiguous
 * ranges, each with private bins, merged at the end by plain addition.
 *
 * Special values (E all ones) are not added; they set bits in *special:
 * bit 0 NaN, bit 1 +infinity, bit 2 -infinity.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_F64 = 0, ORACLE_F32 = 1, ORACLE_BF16 = 2 };

typedef struct {
    const void *x;
    uint64_t begin, end;
    int fmt;
    __int128 bins[2048];
    uint32_t special;
} job_t;

static void accumulate_range(job_t *j)
{
    uint64_t i;
    memset(j->bins, 0, sizeof(j->bins));
    j->special = 0;
    if (j->fmt == ORACLE_F64) {
        const uint64_t *x = (const uint64_t *)j->x;
        for (i = j->begin; i < j->end; ++i) {
            uint64_t b = x[i];
            unsigned e = (unsigned)(b >> 52) & 0x7ffu;
            uint64_t mf = b & ((1ull << 52) - 1);
            int neg = (int)(b >> 63);
            if (e == 0x7ffu) {
                j->special |= mf ? 1u : (neg ? 4u : 2u);
                continue;
            }
            int64_t m = (int64_t)(mf | (e ? (1ull << 52) : 0));
            j->bins[e] += neg ? -(__int128)m : (__int128)m;
        }
    } else {
        /* binary32, or bfloat16 widened to binary32 by a 16-bit shift */
        for (i = j->begin; i < j->end; ++i) {
            uint32_t b;
            if (j->fmt == ORACLE_F32)
                b = ((const uint32_t *)j->x)[i];
            else
                b = (uint32_t)((const uint16_t *)j->x)[i] << 16;
            unsigned e = (b >> 23) & 0xffu;
            uint32_t mf = b & ((1u << 23) - 1);
            int neg = (int)(b >> 31);
            if (e == 0xffu) {
                j->special |= mf ? 1u : (neg ? 4u : 2u);
                continue;
            }
            int64_t m = (int64_t)(mf | (e ? (1u << 23) : 0));
            j->bins[e] += neg ? -(__int128)m : (__int128)m;
        }
    }
}

static void *worker(void *arg)
{
    accumulate_range((job_t *)arg);
    return NULL;
}

/*
 * x: host array of n bit patterns of format fmt.  out_bins: 2048 entries of
 * two int64 words each (low word unsigned, high word signed) holding bin[E].
 * Returns the number of threads used, or -1 on a bad argument or allocation
 * failure.
 */
int oracle_binned_sum(const void *x, uint64_t n, int fmt, int nthreads,
                      int64_t *out_bins, uint32_t *special)
{
    if ((x == NULL && n > 0) || out_bins == NULL || special == NULL)
        return -1;
    if (fmt < ORACLE_F64 || fmt > ORACLE_BF16)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > n / 65536 + 1)
        nthreads = (int)(n / 65536 + 1);
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return -1;
    }
    uint64_t per = n / (uint64_t)nthreads, extra = n % (uint64_t)nthreads, at = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].x = x;
        jobs[t].fmt = fmt;
        jobs[t].begin = at;
        at += per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t].end = at;
    }
    char *running = (char *)calloc((size_t)nthreads, 1);
    if (!running) {
        free(jobs);
        free(tids);
        return -1;
    }
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tids[t], NULL, worker, &jobs[t]) == 0)
            running[t] = 1;
        else
            accumulate_range(&jobs[t]); /* could not start: do it inline */
    }
    accumulate_range(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        if (running[t])
            pthread_join(tids[t], NULL);
    free(running);
    __int128 total[2048];
    memset(total, 0, sizeof(total));
    uint32_t sp = 0;
    for (int t = 0; t < nthreads; ++t) {
        for (int e = 0; e < 2048; ++e)
            total[e] += jobs[t].bins[e];
        sp |= jobs[t].special;
    }
    for (int e = 0; e < 2048; ++e) {
        unsigned __int128 u = (unsigned __int128)total[e];
        out_bins[2 * e] = (int64_t)(uint64_t)u;
        out_bins[2 * e + 1] = (int64_t)(uint64_t)(u >> 64);
    }
    *special = sp;
    free(jobs);
    free(tids);
    return nthreads;
}

/*
 * Per-segment exact sums (many independent sums over one buffer), for
 * checking every segment of a large segmented batch.
 *
 * Segment i holds length[i] elements of format fmt[i] starting byte_off[i]
 * bytes into base.  Each segment is accumulated into exponent bins exactly as
 * above, and its bins are then folded into one wide two's-complement integer
 * in units of 2^-1074 (the fixed-point number of Section 2):
 *
 *     total = sum_E bin[E] * 2^q(E),  q(E) = max(E,1) - 1         (binary64)
 *                                      q(E) = max(E,1) + 924       (binary32)
 *
 * written to out_limbs[i * ORACLE_SEG_LIMBS ...] as little-endian 64-bit
 * limbs.  ORACLE_SEG_LIMBS limbs (2560 bits) hold any total of at most 2^40
 * finite inputs: |total| < 2^40 * 2^1024 * 2^1074.  special[i] gets the
 * special-value bits.  Threads take interleaved segments.
 */
#define ORACLE_SEG_LIMBS 40

typedef struct {
    const uint8_t *base;
    const uint64_t *byte_off, *length;
    const uint32_t *fmt;
    uint64_t nseg, first, stride;
    uint64_t *out_limbs;
    uint32_t *special;
} seg_job_t;

/* limbs += v * 2^s (two's complement over ORACLE_SEG_LIMBS limbs) */
static void add_shifted(uint64_t *limbs, __int128 v, unsigned s)
{
    unsigned k = s / 64, r = s % 64;
    /* v * 2^r as a sign-extended 192-bit value: three limbs */
    unsigned __int128 u = (unsigned __int128)v;
    uint64_t w0 = (uint64_t)(u << r);
    uint64_t w1 = (uint64_t)((u << r) >> 64);
    uint64_t w2 = r ? (uint64_t)(int64_t)(v >> (128 - r)) : (uint64_t)(v < 0 ? -1 : 0);
    uint64_t ext = v < 0 ? ~0ull : 0ull;
    uint64_t carry = 0;
    for (unsigned j = k; j < ORACLE_SEG_LIMBS; ++j) {
        uint64_t add = j == k ? w0 : j == k + 1 ? w1 : j == k + 2 ? w2 : ext;
        unsigned __int128 t = (unsigned __int128)limbs[j] + add + carry;
        limbs[j] = (uint64_t)t;
        carry = (uint64_t)(t >> 64);
    }
}

static void *seg_worker(void *arg)
{
    seg_job_t *j = (seg_job_t *)arg;
    __int128 *bins = (__int128 *)calloc(2048, sizeof(__int128));
    if (!bins)
        return (void *)1;
    for (uint64_t s = j->first; s < j->nseg; s += j->stride) {
        int lo = 2048, hi = -1;
        uint32_t sp = 0;
        const uint64_t n = j->length[s];
        const int fmt = (int)j->fmt[s];
        const uint8_t *p = j->base + j->byte_off[s];
        for (uint64_t i = 0; i < n; ++i) {
            unsigned e;
            int64_t m;
            int neg;
            if (fmt == ORACLE_F64) {
                uint64_t b;
                memcpy(&b, p + 8 * i, 8);
                e = (unsigned)(b >> 52) & 0x7ffu;
                uint64_t mf = b & ((1ull << 52) - 1);
                neg = (int)(b >> 63);
                if (e == 0x7ffu) {
                    sp |= mf ? 1u : (neg ? 4u : 2u);
                    continue;
                }
                m = (int64_t)(mf | (e ? (1ull << 52) : 0));
            } else {
                uint32_t b;
                if (fmt == ORACLE_F32) {
                    memcpy(&b, p + 4 * i, 4);
                } else {
                    uint16_t h;
                    memcpy(&h, p + 2 * i, 2);
                    b = (uint32_t)h << 16;
                }
                e = (b >> 23) & 0xffu;
                uint32_t mf = b & ((1u << 23) - 1);
                neg = (int)(b >> 31);
                if (e == 0xffu) {
                    sp |= mf ? 1u : (neg ? 4u : 2u);
                    continue;
                }
                m = (int64_t)(mf | (e ? (1u << 23) : 0));
            }
            bins[e] += neg ? -(__int128)m : (__int128)m;
            if ((int)e < lo)
                lo = (int)e;
            if ((int)e > hi)
                hi = (int)e;
        }
        uint64_t *limbs = j->out_limbs + s * ORACLE_SEG_LIMBS;
        memset(limbs, 0, ORACLE_SEG_LIMBS * sizeof(uint64_t));
        for (int e = lo; e <= hi; ++e) {
            if (bins[e]) {
                unsigned emin1 = e ? (unsigned)e : 1u;
                unsigned q = fmt == ORACLE_F64 ? emin1 - 1 : emin1 + 924;
                add_shifted(limbs, bins[e], q);
                bins[e] = 0;
            }
        }
        j->special[s] = sp;
    }
    free(bins);
    return NULL;
}

/*
 * Returns the number of threads used, or -1 on a bad argument (an unknown
 * format, a length above 2^40) or allocation failure.
 */
int oracle_segmented_sums(const void *base, const uint64_t *byte_off,
                          const uint64_t *length, const uint32_t *fmt,
                          uint64_t nseg, int nthreads, uint64_t *out_limbs,
                          uint32_t *special)
{
    if (nseg > 0 && (byte_off == NULL || length == NULL || fmt == NULL ||
                     out_limbs == NULL || special == NULL))
        return -1;
    for (uint64_t s = 0; s < nseg; ++s) {
        if (fmt[s] > ORACLE_BF16 || length[s] > (1ull << 40))
            return -1;
        if (length[s] > 0 && base == NULL)
            return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > nseg)
        nthreads = nseg ? (int)nseg : 1;
    seg_job_t *jobs = (seg_job_t *)calloc((size_t)nthreads, sizeof(seg_job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    char *running = (char *)calloc((size_t)nthreads, 1);
    int bad = 0;
    if (!jobs || !tids || !running) {
        free(jobs);
        free(tids);
        free(running);
        return -1;
    }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (seg_job_t){(const uint8_t *)base, byte_off, length, fmt, nseg,
                              (uint64_t)t, (uint64_t)nthreads, out_limbs, special};
    }
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tids[t], NULL, seg_worker, &jobs[t]) == 0)
            running[t] = 1;
        else
            bad |= seg_worker(&jobs[t]) != NULL;
    }
    bad |= seg_worker(&jobs[0]) != NULL;
    for (int t = 1; t < nthreads; ++t) {
        if (running[t]) {
            void *rv = NULL;
            pthread_join(tids[t], &rv);
            bad |= rv != NULL;
        }
    }
    free(jobs);
    free(tids);
    free(running);
    return bad ? -1 : nthreads;
}
