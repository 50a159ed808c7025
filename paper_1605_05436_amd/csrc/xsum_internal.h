// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xsum.h"

namespace xsum {

// What the last block of an accumulation launch does once every block has
// added its digits into the global state.
enum FinishMode : int {
    kKeep = 0,   // carry-normalise the state in place and keep it
    kRound = 1,  // round the state to out_fmt, write out/flags, zero the state
};

struct Finish {
    int mode;
    int out_fmt;       // XSUM_F64 / XSUM_F32 / XSUM_BF16 (resolved, never SAME)
    void *out;         // device, result bit pattern (kRound only)
    uint32_t *flags;   // device, may be null (kRound only)
    int out_slot8;     // nonzero: write the pattern zero-extended to 8 bytes
};

// Launch shape of the single-sum kernel.  blocks == 0 means "one resident
// block per slot the device offers" (persistent grid).
struct Shape {
    int blocks;
};

int element_size(int dtype);

// acc += exact sum of x[0..n), then the finish action.  x must be
// element-aligned.  cu_count is the device's compute-unit count.
hipError_t launch_accumulate(const void *x, uint64_t n, int dtype,
                             xsum_acc_t *acc, const Finish &fin, int cu_count,
                             const Shape &shape, hipStream_t stream);

// Round *acc (unchanged) to out_fmt.
hipError_t launch_finalize(const xsum_acc_t *acc, int out_fmt, void *out,
                           uint32_t *flags, hipStream_t stream);

// *dst += *src, then carry-normalise dst.
hipError_t launch_merge(xsum_acc_t *dst, const xsum_acc_t *src,
                        hipStream_t stream);

// Zero count states with a fill kernel (no memset node, so the call can be
// captured into a graph).
hipError_t launch_zero(xsum_acc_t *acc, uint64_t count, hipStream_t stream);

// Zero `words` 64-bit words with a fill kernel.
hipError_t launch_zero_words(uint64_t *p, uint64_t words, hipStream_t stream);

// Number of blocks a persistent single-sum grid uses for this format.
int persistent_blocks(int dtype, int cu_count);

}  // namespace xsum
