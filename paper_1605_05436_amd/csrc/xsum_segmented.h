// Internal layout of a segmented-sum plan, shared by the planner (host) and
// the segmented kernel (device).
#pragma once

#include <cstddef>

#include <stdint.h>

namespace xsum {

// Copy of one caller descriptor (same layout as xsum_segment_t).
struct SegDesc {
    uint64_t byte_offset;
    uint64_t length;
    uint32_t dtype;
    uint32_t reserved;
};

enum SegTaskKind : uint32_t {
    kLaneGroup = 0,  // up to 64 whole segments, one per lane
    kChunk = 1,      // one chunk of a very long segment, summed by a wave
    kWhole = 2,      // one whole segment, summed and rounded by one wave
};

enum SegChunkFlags : uint32_t {
    kChunkFirst = 1,  // also adds the segment's unaligned head elements
    kChunkLast = 2,   // also adds the segment's ragged tail elements
};
// A lane group's flags field holds log2 of the lanes that share each
// segment in its low three bits (0 to 4: 64 down to 4 segments per group)
// and, in bit 3, whether each lane keeps 8 instead of 16 vectors in flight.
static constexpr uint32_t kLaneGlogMask = 7u;
static constexpr uint32_t kLaneUnroll8 = 8u;

// 32-byte work item.
struct SegTask {
    uint32_t kind_dtype_flags;  // kind | dtype << 8 | flags << 16
    uint32_t a;                 // lane group: first lane entry; else: segment
    uint32_t b;                 // lane group: segment count;  chunk: state slot
    uint32_t nchunks;           // chunk: chunks of its segment
    uint64_t v0;                // whole: byte offset;  chunk: first 16-byte vector
    uint64_t nv;                // whole: elements;     chunk: vectors in the chunk
};

// 16-byte lane entry: the segment one lane of a lane group sums.
struct SegLane {
    uint64_t byte_offset;
    uint32_t length;            // at most the largest lane_max (2^23)
    uint32_t seg;               // output index
};

// Control words at the start of the workspace.  Both return to zero at the
// end of every launch (the last wave to finish resets them).
struct SegCtl {
    uint32_t head;      // next task to pop
    uint32_t done;      // waves that found the queue empty
    uint32_t pad[58];
    uint32_t zero[4];   // always zero: what a lane past its segment's end loads
};

static constexpr uint64_t kSegCtlBytes = sizeof(SegCtl);
static_assert(sizeof(SegCtl) == 256 && offsetof(SegCtl, zero) % 16 == 0,
              "control block: 256 bytes, a 16-byte-aligned zero vector");


// One request chunk list of a serving batch (same layout as xsum_batch_item_t).
struct BatchItem {
    uint64_t ptr;         // device address of the first element
    uint64_t length;      // elements
    uint32_t dtype;
    uint32_t slot;        // destination state
    uint64_t first_task;  // index of the item's first chunk among all tasks
};

}  // namespace xsum
