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

/*
 * Sample the shader clock while other work runs: one single-wave kernel on
 * `stream` takes nsamples samples, one every interval_ticks ticks of the
 * GPU's 100 MHz constant-rate counter, and writes for sample i
 *   out[2i]     the constant-rate counter (100 MHz ticks)
 *   out[2i + 1] the shader-clock counter of the compute unit it runs on,
 * so the shader clock over a sample interval is
 *   (out[2i+3] - out[2i+1]) / (out[2i+2] - out[2i]) * 100 MHz.
 * Launched on a stream of its own before a run of timed launches on another
 * stream, it shows how the clock moves under that load.  The kernel runs for
 * nsamples * interval_ticks / 100 MHz whatever else the GPU does.
 *   out     device, 16 * nsamples bytes, 8-byte aligned
 * XSUM_ERANGE unless nsamples <= 2^20, interval_ticks >= 1 and
 * nsamples * interval_ticks <= 10^9 (10 s); nsamples = 0 is a no-op.
 */
xsum_status_t xsum_probe_clock(uint64_t *out, uint32_t nsamples, uint32_t interval_ticks,
                               void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XSUM_PROBE_H */
