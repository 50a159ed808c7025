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
