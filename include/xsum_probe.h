/*
 * Measurement utilities of libxsum: no part of the summation method.  They
 * give the reference points a benchmark of the exact sum is read against.
 * Same conventions as xsum.h (device pointers, stream as void*, status
 * codes, xsum_last_error()).
 */
#ifndef XSUM_PROBE_H
#define XSUM_PROBE_H

#include <stdint.h>

#include "xsum.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Stream nbytes of device memory at x once, with the access pattern and
 * launch shape of the binary64 single-sum kernel (two-wave workgroups, two
 * per compute unit, 16 non-temporal 16-byte loads per lane in flight, each
 * wave over its own contiguous run), and nothing else: the practical HBM
 * read ceiling of that pattern.  One kernel launch on `stream`.
 *   x       device, 16-byte aligned; nbytes a multiple of 16
 *   sink    device, 4 bytes the kernel may write (so the loads are not
 *           removed); its content is meaningless
 */
xsum_status_t xsum_probe_read(const void *x, uint64_t nbytes, uint32_t *sink, void *stream);

/*
 * Fill nbytes of device memory at buf with the 32-bit value (one kernel
 * launch on `stream`); a buffer larger than the 256 MB last-level cache,
 * filled between timed runs, leaves their input cold.  buf and nbytes must be
 * multiples of 4.
 */
xsum_status_t xsum_probe_flush(void *buf, uint64_t nbytes, uint32_t value, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XSUM_PROBE_H */
