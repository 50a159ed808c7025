// Host-side helpers shared by the C-ABI entry points.
#pragma once

#include "xsum.h"

namespace xsum {

// Output format of a sum: XSUM_SAME means binary64 for binary64 input and
// binary32 for binary32 and bfloat16 input.
inline int resolve_out(int dtype, int out)
{
    if (out == XSUM_SAME)
        return dtype == XSUM_F64 ? XSUM_F64 : XSUM_F32;
    return out;
}

// Bytes of a result in output format out.
inline int out_bytes(int out) { return out == XSUM_F64 ? 8 : out == XSUM_F32 ? 4 : 2; }

}  // namespace xsum
