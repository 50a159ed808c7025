/*
 * xsum: exact summation of IEEE binary floating-point numbers on AMD
 * Instinct MI355X (gfx950), returning the sum rounded once.
 *
 * Method (Goodrich & Eldawy, "Parallel Algorithms for Summing
 * Floating-Point Numbers"): every input is converted to an exact integer
 * representation, the integers are summed without rounding, and the exact
 * total is rounded to a float at the end (Section 1, the problem statement,
 * asks for a faithful rounding of the exact sum).  This library returns the
 * round-to-nearest, ties-to-even result, which is one of the two faithful
 * answers and is unique, so results are bit-reproducible regardless of launch
 * shape, order or batching.
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" must be device memory of the current HIP device
 *    (hipMalloc, or any allocator returning such memory, e.g. PyTorch).  The
 *    caller owns every buffer and every stream it passes; the library keeps no
 *    reference to them after a call returns (asynchronous calls: after the
 *    work completes on the stream).
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *  - Input elements must be aligned to their size (8, 4 or 2 bytes); 16-byte
 *    alignment gives the fastest path.  Any length is accepted, including 0.
 *  - Errors are returned as status codes; no exception crosses the interface.
 *    xsum_last_error() returns a thread-local message for the last failing
 *    call on the calling thread.
 *  - Infinities and NaNs are not errors.  The paper assumes finite inputs;
 *    this library follows IEEE addition for them: a NaN input, or both +inf
 *    and -inf, gives the canonical quiet NaN; otherwise an infinite input
 *    gives that infinity.
 *  - An exact sum of zero is returned as +0.0.  A non-zero exact sum that
 *    rounds beyond the largest finite value returns an infinity of its sign
 *    with XSUM_FLAG_OVERFLOW.
 *  - Calls on distinct streams with distinct workspaces may overlap.
 */
#ifndef XSUM_H
#define XSUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element formats (IEEE 754 binary64, binary32; bfloat16 = upper half of a
 * binary32).  XSUM_SAME as an output format means: binary64 for binary64
 * input, binary32 for binary32 and bfloat16 input. */
typedef enum {
    XSUM_F64 = 0,
    XSUM_F32 = 1,
    XSUM_BF16 = 2,
    XSUM_SAME = 255
} xsum_dtype_t;

typedef enum {
    XSUM_OK = 0,
    XSUM_EINVAL = 1,  /* null pointer, misaligned input, bad size */
    XSUM_EDTYPE = 2,  /* unknown input or output format */
    XSUM_ENOMEM = 3,  /* library-owned allocation failed */
    XSUM_EHIP = 4,    /* a HIP runtime call failed (message has the code) */
    XSUM_ERANGE = 5   /* a size exceeds a documented limit */
} xsum_status_t;

/* Result flags (bitwise OR). */
#define XSUM_FLAG_INEXACT 1u   /* the finite result differs from the exact sum */
#define XSUM_FLAG_OVERFLOW 2u  /* the exact finite sum rounded to +-infinity */
#define XSUM_FLAG_NAN 4u       /* the result is NaN */
#define XSUM_FLAG_INF 8u       /* some input was an infinity */

/* Number of radix-2^32 digits of the exact accumulator.  Digit j weighs
 * 2^(32 j - 1074); digit XSUM_DIGITS-1 is signed and holds the sign. */
#define XSUM_DIGITS 68

/*
 * Exact, mergeable sum state in device memory (Section 2: a superaccumulator
 * of integer digits whose additions need no carry propagation).  576 bytes.
 * `digit` holds the exact sum of everything added so far; `special` records
 * NaN (bit 0), +inf (bit 1) and -inf (bit 2) inputs; `ticket` is used by the
 * library's kernels and must be 0 between calls.  After any xsum call that
 * completes on a state, its digits are in canonical form (digits 0..66 in
 * [0, 2^32), digit 67 in {-1, 0}).  A state is zeroed by xsum_acc_zero, or by
 * a byte-wise zero fill.
 */
typedef struct xsum_acc {
    int64_t digit[XSUM_DIGITS];
    uint32_t special;
    uint32_t ticket;
    uint64_t reserved[3];
} xsum_acc_t;

/* Library version string (static storage). */
const char *xsum_version(void);

/* Thread-local description of the last error on this thread ("" if none). */
const char *xsum_last_error(void);

/*
 * Exact sum of n elements, blocking.
 * Section 3 (steps 2, 5, 6, 7) and Section 5 (scan algorithm when the
 * accumulator fits in fast memory): convert each input to integer digits,
 * add them carry-free, propagate the signed carries once, round once.
 *   x         device, n elements of `dtype`, element-aligned (NULL iff n == 0)
 *   out_dtype XSUM_F64, XSUM_F32, XSUM_BF16 or XSUM_SAME
 *   out_host  host memory receiving the result bit pattern (8, 4 or 2 bytes)
 *   flags_host host, may be NULL; receives XSUM_FLAG_* bits
 * The library keeps one workspace per (device, stream) for this call; it is
 * allocated on first use and kept until process exit.  Returns after the
 * result has been copied to the host.
 */
xsum_status_t xsum_exact_sum(const void *x, uint64_t n, int dtype,
                             int out_dtype, void *out_host,
                             uint32_t *flags_host, void *stream);

/* Convenience: binary64 result of xsum_exact_sum (NaN and a thread-local
 * error message on failure). */
double xsum_exact_sum_f64(const void *x, uint64_t n, int dtype);

/*
 * Exact sum, asynchronous, all in device memory (one kernel launch).
 *   x, n, dtype, out_dtype as for xsum_exact_sum
 *   out_dev   device, receives the result bit pattern (8, 4 or 2 bytes)
 *   flags_dev device, may be NULL; receives XSUM_FLAG_* bits
 *   scratch   device, an xsum_acc_t that is zero (xsum_acc_zero) before the
 *             call; the call leaves it zero again.  Calls sharing a scratch
 *             state must be ordered (same stream, or synchronised).
 * Returns after enqueueing; results are valid when the stream reaches them.
 */
xsum_status_t xsum_exact_sum_async(const void *x, uint64_t n, int dtype,
                                   int out_dtype, void *out_dev,
                                   uint32_t *flags_dev, xsum_acc_t *scratch,
                                   void *stream);

/*
 * xsum_exact_sum_async with an explicit grid size (number of workgroups of
 * the accumulation kernel; 0 = the library's persistent default).  The result
 * does not depend on `blocks`; this exists for tuning and for tests that
 * check exactly that.  blocks < 0 is XSUM_EINVAL.
 */
xsum_status_t xsum_exact_sum_async_blocks(const void *x, uint64_t n,
                                          int dtype, int out_dtype,
                                          void *out_dev, uint32_t *flags_dev,
                                          xsum_acc_t *scratch, int blocks,
                                          void *stream);

/*
 * Accumulator interface (Section 2: two exact states are merged by adding
 * digits; Section 6: reducers' states are combined by a final post-process
 * and rounded once).  All pointers are device pointers; all calls are
 * asynchronous on `stream`.
 */
/* Zero `count` consecutive states. */
xsum_status_t xsum_acc_zero(xsum_acc_t *acc, uint64_t count, void *stream);
/* acc += exact sum of x[0..n).  Leaves acc canonical. */
xsum_status_t xsum_acc_add(xsum_acc_t *acc, const void *x, uint64_t n,
                           int dtype, void *stream);
/* dst += src (exact).  src is unchanged.  Leaves dst canonical. */
xsum_status_t xsum_acc_merge(xsum_acc_t *dst, const xsum_acc_t *src,
                             void *stream);
/* Round the state once to out_dtype (XSUM_SAME means binary64).  acc is
 * unchanged.  out_dev receives 8, 4 or 2 bytes; flags_dev may be NULL. */
xsum_status_t xsum_acc_finalize(const xsum_acc_t *acc, int out_dtype,
                                void *out_dev, uint32_t *flags_dev,
                                void *stream);

/* ------------------------------------------------------------------------
 * Compact encoding of a state (host code only; no device is touched), for
 * checkpoints and for exchanging states between processes (Section 2: a
 * sparse superaccumulator stores only its non-zero components, each with its
 * exponent).  The value is carry-normalised (Section 3, step 6) and written
 * as sign and magnitude; the magnitude is stored as the run of radix-2^32
 * digits from its lowest to its highest non-zero digit.  Little-endian
 * layout: u32 magic 0x31535358 ("XSS1"), u32 special bits, u8 sign (1 =
 * negative), u8 index of the run's first digit (digit j weighs
 * 2^(32 j - 1074)), u8 digit count c, u8 0, then c u32 digits, lowest first:
 * 12 + 4 c bytes, at most XSUM_STATE_ENCODED_MAX.  An all-zero state is the
 * 12-byte header with c = 0.
 * ------------------------------------------------------------------------ */
#define XSUM_STATE_ENCODED_MAX 292

/* Encode a state held in host memory (copy it from the device first; a
 * state copied after any completed xsum call is valid).  Digits may be in any
 * form with |digit| <= 2^62; the value's normalised top digit must lie in
 * [-2^61, 2^61] (every sum of at most 2^31 finite inputs does).  *len
 * receives the encoded size; XSUM_ERANGE if cap is smaller (or buf NULL),
 * with *len still set.  XSUM_EINVAL for NULL acc/len or unknown special bits. */
xsum_status_t xsum_state_encode(const xsum_acc_t *acc, void *buf, size_t cap,
                                size_t *len);

/* Decode into a host state in canonical form (digits 0..66 in [0, 2^32), the
 * signed top digit, special bits, ticket and padding zero); copy it to the
 * device to use it, e.g. as the source of xsum_acc_merge.  XSUM_EINVAL for a
 * wrong magic, length, header field or a digit run that does not start and
 * end with non-zero digits; XSUM_ERANGE for a value outside the encodable
 * range. */
xsum_status_t xsum_state_decode(const void *buf, size_t len, xsum_acc_t *acc);

/* ------------------------------------------------------------------------
 * Inputs in host memory, larger than device memory if need be (Section 5:
 * when the superaccumulator fits in internal memory, one scan that adds the
 * inputs in any order gives the correctly rounded sum; here the device-
 * resident exact state is the internal memory and the host array is read
 * once, in chunks).
 * ------------------------------------------------------------------------ */

/* acc += the exact sum of n elements at x_host (host memory, pageable or
 * pinned; pinned memory is copied at the full host-link rate).  The array is
 * copied in chunks of chunk_bytes (0: 64 MiB; else a multiple of 16 in
 * [4096, 2^34]) into two device staging buffers that alternate, on a copy
 * stream of the call's own, while earlier chunks are added on `stream`.
 * Returns once every chunk has been added (stream synchronised), so x_host
 * may be reused at once.  The staging buffers (at most 2 x chunk_bytes of
 * device memory) are allocated and freed by the call.  Errors: as
 * xsum_acc_add, XSUM_ERANGE for a bad chunk_bytes, XSUM_ENOMEM if staging
 * cannot be allocated. */
xsum_status_t xsum_acc_add_host(xsum_acc_t *acc, const void *x_host, uint64_t n,
                                int dtype, uint64_t chunk_bytes, void *stream);

/* Exact sum of n elements in host memory, rounded once to out_dtype
 * (XSUM_SAME: binary64 for binary64 input, else binary32), written to
 * out_host (8, 4 or 2 bytes) with flags to flags_host (may be NULL).
 * Blocking; allocates a 576-byte state plus the staging buffers of
 * xsum_acc_add_host for the duration of the call. */
xsum_status_t xsum_exact_sum_host(const void *x_host, uint64_t n, int dtype,
                                  int out_dtype, void *out_host, uint32_t *flags_host,
                                  uint64_t chunk_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Condition-number-sensitive sum (Section 4): the input is summed with
 * r-truncated sparse superaccumulators up a summation tree, the root is
 * tested, and r is squared (2, 4, 16) until the test passes.  r = 256 would
 * exceed the 68 digit positions, so that pass truncates nothing and is the
 * exact sum itself.  The test certifies the round-to-nearest-even result (the
 * same bits and flags as xsum_exact_sum), not only a faithful one.
 * ------------------------------------------------------------------------ */

#define XSUM_TRUNC_MAX_R 16

/* Root of one truncated pass (device memory, written by the pass).
 *   index/value  the root's entries, most significant first: `count` of
 *                them, each worth value * 2^(32 index - 1074); value is the
 *                exact integer sum of the radix-2^32 digits added at that
 *                index (not carry-normalised).  Unused entries have a
 *                negative index and value 0.
 *   bound_index/bound_value  everything truncated anywhere on the tree sums
 *                to at most bound_value * 2^(32 bound_index - 1074) in
 *                magnitude; bound_value 0 means nothing was lost.
 *   special      NaN (bit 0), +inf (bit 1), -inf (bit 2) inputs seen.
 *   certified    1: bits/flags hold the round-to-nearest-even sum (bit
 *                pattern zero-extended to 64 bits); 0: the pass cannot tell.
 *   r            the truncation parameter of the pass. */
typedef struct xsum_trunc_root {
    int32_t index[XSUM_TRUNC_MAX_R];
    int64_t value[XSUM_TRUNC_MAX_R];
    uint32_t count;
    int32_t bound_index;
    uint64_t bound_value;
    uint32_t special;
    uint32_t certified;
    uint64_t bits;
    uint32_t flags;
    uint32_t r;
} xsum_trunc_root_t;

/* Device workspace bytes of the calls below (fixed, about 0.5 MiB). */
size_t xsum_truncated_workspace_size(void);

/*
 * One pass with truncation parameter r (2, 4 or 16), asynchronous, one
 * kernel launch (Section 4, the bottom-up merge-and-sum with r-truncated
 * sparse superaccumulators, Lemma 3 for each pairwise sum, and the stopping
 * test on the root).
 *   x, n, dtype, out_dtype  as for xsum_exact_sum; n <= 2^31 (XSUM_ERANGE)
 *   root_dev   device, receives the pass's xsum_trunc_root_t
 *   workspace  device, 256-byte aligned, xsum_truncated_workspace_size()
 *              bytes, zero-filled before its first use; every pass leaves
 *              it as it found it.  Calls sharing a workspace must be ordered.
 * The record does not depend on scheduling: the tree's shape is fixed by n,
 * the input's address, the device's compute-unit count and how many blocks
 * of the pass's kernel fit one compute unit (a property of the build).
 */
xsum_status_t xsum_truncated_round(const void *x, uint64_t n, int dtype, int out_dtype,
                                   int r, xsum_trunc_root_t *root_dev, void *workspace,
                                   size_t ws_bytes, void *stream);

/*
 * The whole iteration, blocking: passes with r = 2, 4, 16 until one is
 * certified, else the untruncated pass (the exact-sum kernel).  Writes the
 * result bit pattern to out_host (8, 4 or 2 bytes), flags to flags_host (may
 * be NULL) and the r of the certifying pass to r_host (may be NULL; 0 when the
 * untruncated pass gave the result).  The result equals xsum_exact_sum's.
 * workspace as for xsum_truncated_round; the call zero-fills it first.  Reads
 * each pass's record back, so it cannot be captured into a graph.
 */
xsum_status_t xsum_exact_sum_truncated(const void *x, uint64_t n, int dtype, int out_dtype,
                                       void *out_host, uint32_t *flags_host, int *r_host,
                                       void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Segmented sums: many independent exact sums of uneven lengths and mixed
 * formats in one persistent kernel launch (Section 6: each reducer sums its
 * own inputs into a superaccumulator; long inputs are summed per chunk and
 * the chunk states merged and rounded once).
 * ------------------------------------------------------------------------ */

/* One segment: `length` elements of format `dtype` starting `byte_offset`
 * bytes after the run's base pointer.  byte_offset must be a multiple of the
 * element size.  Same layout on host and device (24 bytes). */
typedef struct xsum_segment {
    uint64_t byte_offset;
    uint64_t length;
    uint32_t dtype;     /* XSUM_F64, XSUM_F32 or XSUM_BF16 */
    uint32_t reserved;  /* ignored */
} xsum_segment_t;

/* Tuning knobs of a plan, indexed by dtype d where per-format; 0 in any
 * field means the library default.
 *   lane_max[d]   segments with at most this many elements are summed by a
 *                 few lanes each, 16 to 64 segments to a wave (default 16384 /
 *                 16384 / 32768 for binary64 / binary32 / bfloat16: 128 KiB of
 *                 binary64, 64 KiB of the narrow formats; at most 2^20 / 2^22
 *                 / 2^23)
 *   wave_max[d]   longer segments with at most this many elements are summed
 *                 whole by one wave (default: 1 MiB of input for binary64,
 *                 4 MiB for binary32 and bfloat16; values above 2^36 act as
 *                 2^36)
 *   chunk_vectors longer segments still are cut into chunks of this many
 *                 16-byte vectors, summed by separate waves whose states are
 *                 merged (default 2^16 = 1 MiB, range [64, 2^26])
 *   blocks_per_cu resident one-wave workgroups per compute unit (default 4,
 *                 range [1, 16])
 *   lane_buckets  per-lane segments are grouped by length in this many
 *                 buckets per doubling (default 4, at most 64) and taken in
 *                 buffer order inside a bucket
 *   two_lanes_from, four_lanes_from
 *                 segment sizes in bytes from which a segment summed in a lane
 *                 group gets two, then four lanes (default 2048 and 32768;
 *                 four_lanes_from below two_lanes_from is XSUM_ERANGE)
 *   lanes[d][b]   per format d and size bucket b (lane-group segments of
 *                 2^b to 2^(b+1) - 1 bytes; bucket 0 also holds empty ones,
 *                 bucket 23 everything larger): the lanes each segment gets,
 *                 1, 2, 4, 8 or 16 (0: as two_lanes_from / four_lanes_from
 *                 decide; other values are XSUM_ERANGE)
 *   lane_unroll[d][b]
 *                 per format and size bucket: 16-byte vectors each lane has
 *                 in flight per step, 8 or 16 (0: 16)
 * Every tuning gives the same result bits; only the speed differs. */
#define XSUM_TUNE_BUCKETS 24
typedef struct xsum_seg_tuning {
    uint64_t lane_max[3];
    uint64_t wave_max[3];
    uint64_t chunk_vectors;
    uint32_t blocks_per_cu;
    uint32_t lane_buckets;
    uint64_t two_lanes_from;
    uint64_t four_lanes_from;
    uint8_t lanes[3][XSUM_TUNE_BUCKETS];
    uint8_t lane_unroll[3][XSUM_TUNE_BUCKETS];
} xsum_seg_tuning_t;

/* Plan statistics. */
typedef struct xsum_plan_info {
    uint64_t nseg, lane_segments, wave_segments, chunked_segments, chunks,
        work_items;
    uint64_t lane_max[3], wave_max[3], chunk_vectors, workspace_bytes;
    uint32_t blocks, reserved;
} xsum_plan_info_t;

typedef struct xsum_plan xsum_plan_t;  /* opaque, owned by the library */

/*
 * Build a plan from host descriptors (copied; the caller may free them).
 * Segments are bucketed by format and length: short ones are grouped 64 to a
 * wave, one per lane, longest first; longer ones get a wave each; the longest
 * are cut into chunks, each such segment with a state slot in the workspace.
 * The plan lives on the current device.
 *   out_dtype  XSUM_SAME (binary64 for binary64 segments, binary32 for the
 *              others) or one output format for every segment
 *   tuning     may be NULL
 * Errors: XSUM_EINVAL (NULL pointers, misaligned offsets), XSUM_EDTYPE,
 * XSUM_ERANGE (more than 2^31-1 segments, a length above 2^40, bad tuning),
 * XSUM_ENOMEM / XSUM_EHIP.
 */
xsum_status_t xsum_segmented_plan(const xsum_segment_t *segs_host,
                                  uint64_t nseg, int out_dtype,
                                  const xsum_seg_tuning_t *tuning,
                                  xsum_plan_t **plan);
void xsum_plan_destroy(xsum_plan_t *plan);
xsum_status_t xsum_plan_get_info(const xsum_plan_t *plan,
                                 xsum_plan_info_t *info);

/* Bytes of device workspace a run of this plan needs (control words plus one
 * 576-byte state per chunked segment). */
size_t xsum_plan_workspace_size(const xsum_plan_t *plan);

/* Zero a workspace (a fill kernel on `stream`, no memset).  Needed once after
 * allocation; every completed run leaves the workspace zeroed again.
 * ws_bytes must be a multiple of 8. */
xsum_status_t xsum_segmented_workspace_init(void *workspace, size_t ws_bytes,
                                            void *stream);

/*
 * Run a plan: one kernel launch on `stream`, asynchronous.
 *   base       device, 16-byte aligned; segment i starts at base + offset_i
 *   out        device, nseg 8-byte slots; slot i receives segment i's result
 *              bit pattern zero-extended to 64 bits
 *   flags      device, nseg uint32 (XSUM_FLAG_* per segment), may be NULL
 *   workspace  device, >= xsum_plan_workspace_size(plan) bytes, zeroed
 *              once by xsum_segmented_workspace_init; runs sharing a
 *              workspace must be ordered
 * The launch contains no memset and no host synchronisation, so it may be
 * captured into a graph and replayed.
 */
xsum_status_t xsum_segmented_run(const xsum_plan_t *plan, const void *base,
                                 void *out, uint32_t *flags, void *workspace,
                                 size_t ws_bytes, void *stream);

/*
 * xsum_segmented_run for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid it): the
 * workspace is a 1 MiB array that the library holds on each device until the
 * process ends, so the caller passes only the plan, inputs and outputs.  The
 * call allocates nothing; it clears the part of the array the plan uses with
 * a fill kernel and launches the run, both on `stream`.
 *   plan        its xsum_plan_workspace_size must be at most 1 MiB (control
 *               words plus at most 1820 chunked segments), else XSUM_ERANGE
 *   base, out, flags, stream as for xsum_segmented_run
 * Every call on one device shares that device's array: calls that overlap
 * (on different streams, or from different threads) race and give wrong
 * results; order them.
 */
xsum_status_t xsum_segmented_run_noalloc(const xsum_plan_t *plan, const void *base,
                                         void *out, uint32_t *flags, void *stream);

/* Capture one xsum_segmented_run into an instantiated HIP graph (returned as
 * hipGraphExec_t in *graph_exec); replay it with xsum_graph_launch. */
xsum_status_t xsum_segmented_capture(const xsum_plan_t *plan, const void *base,
                                     void *out, uint32_t *flags,
                                     void *workspace, size_t ws_bytes,
                                     void **graph_exec);
xsum_status_t xsum_graph_launch(void *graph_exec, void *stream);
void xsum_graph_destroy(void *graph_exec);

/*
 * One-shot segmented sums (Section 1's problem, once per segment; Section 6:
 * each segment is a reducer's key, summed into its own superaccumulator and
 * rounded once), without a plan object: the call plans with the default
 * tuning, puts the plan in the caller's workspace and launches.
 *   base       device, 16-byte aligned; segment i starts at base + offset_i
 *   segs       nseg descriptors, in device or host memory
 *   out_dtype  XSUM_SAME (binary64 for binary64 segments, binary32 for the
 *              others) or one output format for every segment
 *   out        device, nseg 8-byte slots (result bit pattern, zero-extended)
 *   flags      device, nseg uint32, may be NULL
 *   workspace  device, 256-byte aligned, at least
 *              xsum_segmented_workspace_size(nseg, total elements) bytes (or
 *              the exact need of this table, named in the error message); no
 *              initialisation needed, the call zeroes what must start at zero
 * Blocking on the host until the plan is in the workspace: it first waits
 * for the work already queued on `stream` (which may produce the table or
 * still use the workspace), then reads the table; the sums themselves run
 * asynchronously on `stream`.  Not capturable into a graph (it
 * synchronises); use xsum_segmented_plan + xsum_segmented_capture for
 * repeated batches of the same shape, which also skips the planning.
 * Errors: as xsum_segmented_plan, plus XSUM_EINVAL for NULL or misaligned
 * pointers and a workspace that is too small.  nseg == 0 does nothing.
 */
xsum_status_t xsum_exact_sum_segmented(const void *base, const xsum_segment_t *segs,
                                       uint64_t nseg, int out_dtype, void *out,
                                       uint32_t *flags, void *workspace, size_t ws_bytes,
                                       void *stream);

/* Workspace bytes that suffice for xsum_exact_sum_segmented on any table of
 * nseg segments holding total_elems elements in all (an upper bound: control
 * words, one state per possible chunked segment, the segment table, the
 * largest possible number of work items and the lane entries).  0 if nseg >=
 * 2^31 or total_elems > 2^50. */
size_t xsum_segmented_workspace_size(uint64_t nseg, uint64_t total_elems);

/* ------------------------------------------------------------------------
 * Serving batches: one launch adds chunks of many requests into per-request
 * device states that persist across launches (continuous batching); a second
 * launch rounds the states of the requests that are complete.  This is
 * Section 6's combine / reduce / post-process with the reducer state kept
 * between launches: chunks of one request are combined into its
 * superaccumulator by exact integer addition in any order and batch, and the
 * post-process rounds it once, so a request's result does not depend on the
 * batches it was cut into or the requests it shared them with.
 * ------------------------------------------------------------------------ */

/* One request's contribution to a batch (32 bytes, in device memory).
 *   ptr         device address of the first element, element-aligned
 *   length      elements
 *   dtype       XSUM_F64, XSUM_F32 or XSUM_BF16
 *   slot        index of the destination xsum_acc_t in `states`
 *   first_task  sum of xsum_batch_item_tasks() over the preceding items
 * Items must be ordered by first_task; they are trusted as given. */
typedef struct xsum_batch_item {
    uint64_t ptr;
    uint64_t length;
    uint32_t dtype;
    uint32_t slot;
    uint64_t first_task;
} xsum_batch_item_t;

/* Number of work items (chunks of chunk_vectors 16-byte vectors) that one
 * batch item takes; at least 1.  Host function, no device access. */
uint64_t xsum_batch_item_tasks(uint64_t ptr, uint64_t length, int dtype,
                               uint64_t chunk_vectors);

/*
 * states[item.slot] += exact sum of the item's elements, for every item, in
 * one persistent launch on `stream`.  Items sharing a slot are all added.
 *   items        device array of nitems items
 *   ntasks       total work items (sum of xsum_batch_item_tasks), < 2^32
 *   chunk_vectors the value used for xsum_batch_item_tasks, in [64, 2^26]
 *   states       device states; a state may take at most 2^20 batches
 *                between two finalizations
 *   ctl          device, 256 bytes, zeroed once before first use; every
 *                completed launch leaves it zeroed.  Launches sharing ctl
 *                must be ordered.
 */
xsum_status_t xsum_batch_add(const xsum_batch_item_t *items, uint32_t nitems,
                             uint64_t ntasks, uint64_t chunk_vectors,
                             xsum_acc_t *states, void *ctl, void *stream);

/*
 * For i < n: round states[slots[i]] once to fmts[i] (XSUM_F64/F32/BF16), write
 * the bit pattern zero-extended into out[i] (8-byte slots) and the flags into
 * flags[i] (may be NULL), then zero the state.  One launch on `stream`.
 */
xsum_status_t xsum_batch_finalize(const uint32_t *slots, const uint32_t *fmts,
                                  uint32_t n, xsum_acc_t *states, void *out,
                                  uint32_t *flags, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XSUM_H */
