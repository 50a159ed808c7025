// Host side of segmented sums: planning (bucketing segments into per-lane
// groups and per-wave chunks), workspace sizing, launch and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "xsum.h"
#include "xsum_internal.h"
#include "xsum_segmented.h"

namespace xsum {
hipError_t launch_segmented(const void *base, const SegDesc *segs,
                            const SegTask *tasks, uint32_t ntasks,
                            const SegLane *lanes, xsum_acc_t *states,
                            SegCtl *ctl, int out_mode, uint64_t *out,
                            uint32_t *flags, int blocks, hipStream_t stream);
int segmented_blocks(int cu_count, int blocks_per_cu);
uint64_t segmented_chunk_vectors();
xsum_status_t api_fail(xsum_status_t st, const std::string &msg);
xsum_status_t api_hip_fail(hipError_t e, const char *what);
xsum_status_t api_current_cus(int *dev, int *cus);
hipError_t launch_batch_add(const BatchItem *items, uint32_t nitems,
                            uint64_t ntasks, uint64_t chunk_vectors,
                            xsum_acc_t *states, SegCtl *ctl, int blocks,
                            hipStream_t stream);
hipError_t launch_batch_finalize(const uint32_t *slots, const uint32_t *fmts,
                                 uint32_t n, xsum_acc_t *states, uint64_t *out,
                                 uint32_t *flags, hipStream_t stream);
}  // namespace xsum

// Workspace of xsum_segmented_run_noalloc: one array per device, held until
// the process ends.  Host code never uses this name as an address (on the
// host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device.
static constexpr size_t kNoallocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

struct xsum_plan {
    int device = 0;
    uint64_t nseg = 0;
    int out_mode = XSUM_SAME;
    xsum::SegDesc *d_segs = nullptr;
    xsum::SegTask *d_tasks = nullptr;
    xsum::SegLane *d_lanes = nullptr;
    uint32_t ntasks = 0, nslots = 0;
    int blocks = 0;
    xsum_plan_info_t info{};
};

namespace {

using xsum::api_fail;
using xsum::api_hip_fail;

constexpr int kPerVec[3] = {2, 4, 8};
constexpr int kBytes[3] = {8, 4, 2};
// Default per-lane limits: segments up to this many elements are summed by
// lane groups (128 KiB of binary64, 64 KiB of the narrow formats; binary64
// segments of 64-128 KiB measured about 1% faster there than as whole-wave
// items).
constexpr uint64_t kLaneMaxDefault[3] = {16384, 16384, 32768};
// segment sizes (bytes) from which lane groups give a segment two or four lanes
constexpr uint64_t kTwoLanesFromDefault = 2048, kFourLanesFromDefault = 32768;
// Segments up to 1 MiB (binary64) or 4 MiB (binary32, bfloat16) are summed
// whole by one wave; longer ones are cut into chunks (1 MiB by default) that
// neighbouring waves take at about the same time.  Measured on the binary64
// segments of 10^6 lognormal lengths: 1-4 MiB segments summed whole, each by
// its own wave over a region of its own, stream at about 3.8 TB/s; as 1 MiB
// chunks at about 5.3 TB/s.  The narrow formats' batch did not gain.
constexpr uint64_t kWaveMaxDefault[3] = {1ull << 17, 1ull << 20, 1ull << 21};

void free_plan(xsum_plan *p)
{
    if (!p)
        return;
    if (p->d_segs)
        (void)hipFree(p->d_segs);
    if (p->d_tasks)
        (void)hipFree(p->d_tasks);
    if (p->d_lanes)
        (void)hipFree(p->d_lanes);
    delete p;
}

// A plan as built on the host, before its arrays are placed in device memory.
struct HostPlan {
    std::vector<xsum::SegTask> tasks;
    std::vector<xsum::SegLane> lanes;
    uint32_t nslots = 0;
    int blocks = 0;
    xsum_plan_info_t info{};
};

xsum_status_t make_plan(const xsum_segment_t *segs, uint64_t nseg, int out_dtype,
                        const xsum_seg_tuning_t *tuning, int cus, HostPlan &hp)
{
    if (nseg > 0 && segs == nullptr)
        return api_fail(XSUM_EINVAL, "segment array is NULL with nseg > 0");
    if (nseg >= (1ull << 31))
        return api_fail(XSUM_ERANGE, "at most 2^31 - 1 segments per plan");
    if (!(out_dtype == XSUM_SAME || out_dtype == XSUM_F64 || out_dtype == XSUM_F32 ||
          out_dtype == XSUM_BF16))
        return api_fail(XSUM_EDTYPE, "unknown output dtype " + std::to_string(out_dtype));
    uint64_t lane_max[3], wave_max[3];
    for (int d = 0; d < 3; ++d) {
        lane_max[d] = kLaneMaxDefault[d];
        wave_max[d] = kWaveMaxDefault[d];
    }
    uint64_t chunk_vectors = xsum::segmented_chunk_vectors();
    int blocks_per_cu = 0;
    int lane_buckets = 4;
    uint64_t two_lanes_from = kTwoLanesFromDefault, four_lanes_from = kFourLanesFromDefault;
    if (tuning) {
        if (tuning->two_lanes_from)
            two_lanes_from = tuning->two_lanes_from;
        if (tuning->four_lanes_from)
            four_lanes_from = tuning->four_lanes_from;
        if (four_lanes_from < two_lanes_from)
            return api_fail(XSUM_ERANGE, "four_lanes_from below two_lanes_from");
        if (tuning->lane_buckets)
            lane_buckets = (int)tuning->lane_buckets;
        if (lane_buckets > 64)
            return api_fail(XSUM_ERANGE, "lane_buckets above 64");
        for (int d = 0; d < 3; ++d) {
            if (tuning->lane_max[d])
                lane_max[d] = tuning->lane_max[d];
            if (tuning->wave_max[d])
                wave_max[d] = tuning->wave_max[d];
        }
        if (tuning->chunk_vectors)
            chunk_vectors = tuning->chunk_vectors;
        for (int d = 0; d < 3; ++d)
            for (int b = 0; b < XSUM_TUNE_BUCKETS; ++b) {
                const uint8_t g = tuning->lanes[d][b], u = tuning->lane_unroll[d][b];
                if (g > 16 || (g & (g - 1)) != 0)
                    return api_fail(XSUM_ERANGE, "lanes per segment must be 1, 2, 4, 8 or 16");
                if (u != 0 && u != 8 && u != 16)
                    return api_fail(XSUM_ERANGE, "lane_unroll must be 8 or 16");
            }
        blocks_per_cu = (int)tuning->blocks_per_cu;
        if (lane_max[0] > (1u << 20) || lane_max[1] > (1u << 22) || lane_max[2] > (1u << 23))
            return api_fail(XSUM_ERANGE, "lane_max too large");
        // one wave sums a segment of up to wave_max elements: at most 2^30
        // per lane keeps every binned column entry below 2^62
        for (int d = 0; d < 3; ++d)
            if (wave_max[d] > (uint64_t(1) << 36))
                wave_max[d] = uint64_t(1) << 36;
        if (chunk_vectors < 64 || chunk_vectors > (1u << 26))
            return api_fail(XSUM_ERANGE, "chunk_vectors out of range [64, 2^26]");
        if (blocks_per_cu < 0 || blocks_per_cu > 16)
            return api_fail(XSUM_ERANGE, "blocks_per_cu out of range [0, 16]");
    }
    // validate descriptors, split into per-lane, per-wave and chunked segments
    std::vector<uint32_t> lane_ids[3];
    std::vector<uint32_t> wave_ids;
    std::vector<uint32_t> chunk_ids;
    for (uint64_t i = 0; i < nseg; ++i) {
        const uint32_t dt = segs[i].dtype;
        if (dt > 2)
            return api_fail(XSUM_EDTYPE, "segment " + std::to_string(i) + ": unknown dtype");
        if (segs[i].byte_offset % (uint64_t)kBytes[dt] != 0)
            return api_fail(XSUM_EINVAL, "segment " + std::to_string(i) +
                                             ": offset not aligned to its element size");
        if (segs[i].length > (1ull << 40))
            return api_fail(XSUM_ERANGE, "segment " + std::to_string(i) + ": length above 2^40");
        if (segs[i].length <= lane_max[dt])
            lane_ids[dt].push_back((uint32_t)i);
        else if (segs[i].length <= wave_max[dt])
            wave_ids.push_back((uint32_t)i);
        else
            chunk_ids.push_back((uint32_t)i);
    }
    struct HostTask {
        xsum::SegTask t;
        uint64_t cost;  // estimated time: vectors one lane walks through
    };
    std::vector<HostTask> tasks;
    std::vector<xsum::SegLane> lanes;
    // long segments: chunks of chunk_vectors 16-byte vectors, one state each
    uint32_t slots = 0;
    uint64_t nchunks_total = 0;
    for (uint32_t id : chunk_ids) {
        const uint32_t dt = segs[id].dtype;
        const uint64_t L = segs[id].length;
        uint64_t head = ((16 - (segs[id].byte_offset & 15)) & 15) / kBytes[dt];
        if (head > L)
            head = L;
        const uint64_t nvs = (L - head) / kPerVec[dt];
        uint64_t nch = (nvs + chunk_vectors - 1) / chunk_vectors;
        if (nch == 0)
            nch = 1;
        if (nch >= (1ull << 32))
            return api_fail(XSUM_ERANGE, "too many chunks in one segment");
        for (uint64_t c = 0; c < nch; ++c) {
            HostTask h{};
            uint32_t fl = (c == 0 ? xsum::kChunkFirst : 0) | (c + 1 == nch ? xsum::kChunkLast : 0);
            h.t.kind_dtype_flags = xsum::kChunk | (dt << 8) | (fl << 16);
            h.t.a = id;
            h.t.b = slots;
            h.t.nchunks = (uint32_t)nch;
            h.t.v0 = c * chunk_vectors;
            h.t.nv = std::min(chunk_vectors, nvs - std::min(nvs, c * chunk_vectors));
            h.cost = h.t.nv / 64 + 1;
            tasks.push_back(h);
        }
        nchunks_total += nch;
        ++slots;
    }
    // longer segments: one wave each
    for (uint32_t id : wave_ids) {
        const uint32_t dt = segs[id].dtype;
        HostTask h{};
        h.t.kind_dtype_flags = xsum::kWhole | (dt << 8);
        h.t.a = id;
        h.t.v0 = segs[id].byte_offset;
        h.t.nv = segs[id].length;
        h.cost = segs[id].length / kPerVec[dt] / 64 + 1;
        tasks.push_back(h);
    }
    // short segments, 64 per lane group: bucketed by length (lane_buckets
    // buckets per doubling, longest bucket first) so a group's lanes finish
    // together, and in buffer order inside a bucket so a group's 64 streams
    // stay close in memory (few distinct pages per load instruction)
    for (int dt = 0; dt < 3; ++dt) {
        std::vector<uint32_t> &ids = lane_ids[dt];
        auto bucket = [&](uint32_t id) -> int {
            const uint64_t L = segs[id].length;
            if (L == 0)
                return -1;
            int b = 63 - __builtin_clzll(L);          // floor(log2 L)
            if (lane_buckets <= 1)
                return b;
            // fractional part of log2 L from the bits below the leading one
            const uint64_t frac = b >= 8 ? (L >> (b - 8)) & 0xff : (L << (8 - b)) & 0xff;
            return b * lane_buckets + (int)((frac * (uint64_t)lane_buckets) >> 8);
        };
        std::stable_sort(ids.begin(), ids.end(), [&](uint32_t x, uint32_t y) {
            const int bx = bucket(x), by = bucket(y);
            if (bx != by)
                return bx > by;
            return segs[x].byte_offset < segs[y].byte_offset;
        });
        for (size_t g = 0; g < ids.size();) {
            // lanes per segment: one for short segments (the per-group
            // rounding is then shared by 64 segments), two or four for longer
            // ones, whose loads then touch fewer, longer runs of memory
            const uint64_t bytes0 = segs[ids[g]].length * kBytes[dt];
            uint32_t glog = bytes0 < two_lanes_from ? 0 : bytes0 < four_lanes_from ? 1 : 2;
            uint32_t unroll8 = 0;
            if (tuning) {
                const int sb = bytes0 ? std::min(63 - __builtin_clzll(bytes0),
                                                 XSUM_TUNE_BUCKETS - 1) : 0;
                if (tuning->lanes[dt][sb])
                    glog = (uint32_t)__builtin_ctz(tuning->lanes[dt][sb]);
                if (tuning->lane_unroll[dt][sb] == 8)
                    unroll8 = xsum::kLaneUnroll8;
            }
            const size_t cnt = std::min<size_t>(64u >> glog, ids.size() - g);
            HostTask h{};
            h.t.kind_dtype_flags = xsum::kLaneGroup | ((uint32_t)dt << 8) |
                                   ((glog | unroll8) << 16);
            h.t.a = (uint32_t)lanes.size();
            h.t.b = (uint32_t)cnt;
            uint64_t maxlen = 0;
            for (size_t k = g; k < g + cnt; ++k)
                maxlen = std::max<uint64_t>(maxlen, segs[ids[k]].length);
            h.cost = (maxlen / kPerVec[dt] >> glog) + 1;
            tasks.push_back(h);
            for (size_t k = g; k < g + cnt; ++k)
                lanes.push_back({segs[ids[k]].byte_offset, (uint32_t)segs[ids[k]].length, ids[k]});
            g += cnt;
        }
    }
    // longest work first, so the queue drains evenly
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const HostTask &x, const HostTask &y) { return x.cost > y.cost; });
    // the queue counter runs past the last item by a few claims per wave
    if (tasks.size() >= (1ull << 31))
        return api_fail(XSUM_ERANGE, "too many work items");

    hp.nslots = slots;
    hp.blocks = xsum::segmented_blocks(cus, blocks_per_cu);
    hp.info.nseg = nseg;
    hp.info.lane_segments = lane_ids[0].size() + lane_ids[1].size() + lane_ids[2].size();
    hp.info.wave_segments = wave_ids.size();
    hp.info.chunked_segments = chunk_ids.size();
    hp.info.chunks = nchunks_total;
    hp.info.work_items = tasks.size();
    hp.info.blocks = (uint32_t)hp.blocks;
    for (int d = 0; d < 3; ++d) {
        hp.info.lane_max[d] = lane_max[d];
        hp.info.wave_max[d] = wave_max[d];
    }
    hp.info.chunk_vectors = chunk_vectors;
    hp.info.workspace_bytes = xsum::kSegCtlBytes + (uint64_t)slots * sizeof(xsum_acc_t);

    hp.tasks.resize(tasks.size());
    for (size_t i = 0; i < tasks.size(); ++i)
        hp.tasks[i] = tasks[i].t;
    hp.lanes = std::move(lanes);
    return XSUM_OK;
}

// Where the one-shot call puts a plan in the caller's workspace: control
// words, chunk states, then the segment table, work items and lane entries,
// each on a 256-byte boundary.
struct OneshotLayout {
    uint64_t segs, tasks, lanes, total;
};

OneshotLayout oneshot_layout(uint64_t nseg, uint64_t ntasks, uint64_t nlanes, uint64_t nslots)
{
    auto up = [](uint64_t v) { return (v + 255) & ~uint64_t(255); };
    OneshotLayout L;
    L.segs = up(xsum::kSegCtlBytes + nslots * sizeof(xsum_acc_t));
    L.tasks = up(L.segs + nseg * sizeof(xsum::SegDesc));
    L.lanes = up(L.tasks + ntasks * sizeof(xsum::SegTask));
    L.total = L.lanes + nlanes * sizeof(xsum::SegLane);
    return L;
}

}  // namespace

extern "C" {

xsum_status_t xsum_segmented_plan(const xsum_segment_t *segs, uint64_t nseg,
                                  int out_dtype, const xsum_seg_tuning_t *tuning,
                                  xsum_plan_t **plan_out)
{
    if (plan_out == nullptr)
        return api_fail(XSUM_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    int dev, cus;
    xsum_status_t st = xsum::api_current_cus(&dev, &cus);
    if (st != XSUM_OK)
        return st;
    HostPlan hp;
    st = make_plan(segs, nseg, out_dtype, tuning, cus, hp);
    if (st != XSUM_OK)
        return st;
    xsum_plan *p = new xsum_plan();
    p->device = dev;
    p->nseg = nseg;
    p->out_mode = out_dtype;
    p->ntasks = (uint32_t)hp.tasks.size();
    p->nslots = hp.nslots;
    p->blocks = hp.blocks;
    p->info = hp.info;
    const std::vector<xsum::SegTask> &flat = hp.tasks;
    const std::vector<xsum::SegLane> &lanes = hp.lanes;
    hipError_t e = hipSuccess;
    if (nseg)
        e = hipMalloc((void **)&p->d_segs, nseg * sizeof(xsum::SegDesc));
    if (e == hipSuccess && !flat.empty())
        e = hipMalloc((void **)&p->d_tasks, flat.size() * sizeof(xsum::SegTask));
    if (e == hipSuccess && !lanes.empty())
        e = hipMalloc((void **)&p->d_lanes, lanes.size() * sizeof(xsum::SegLane));
    if (e == hipSuccess && nseg)
        e = hipMemcpy(p->d_segs, segs, nseg * sizeof(xsum::SegDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess && !flat.empty())
        e = hipMemcpy(p->d_tasks, flat.data(), flat.size() * sizeof(xsum::SegTask),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !lanes.empty())
        e = hipMemcpy(p->d_lanes, lanes.data(), lanes.size() * sizeof(xsum::SegLane),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_plan(p);
        return e == hipErrorOutOfMemory ? api_fail(XSUM_ENOMEM, "plan allocation failed")
                                        : api_hip_fail(e, "plan upload");
    }
    *plan_out = p;
    return XSUM_OK;
}

void xsum_plan_destroy(xsum_plan_t *plan) { free_plan(plan); }

xsum_status_t xsum_plan_get_info(const xsum_plan_t *plan, xsum_plan_info_t *info)
{
    if (plan == nullptr || info == nullptr)
        return api_fail(XSUM_EINVAL, "plan or info is NULL");
    *info = plan->info;
    return XSUM_OK;
}

size_t xsum_plan_workspace_size(const xsum_plan_t *plan)
{
    return plan ? (size_t)plan->info.workspace_bytes : 0;
}

size_t xsum_segmented_workspace_size(uint64_t nseg, uint64_t total_elems)
{
    // With the default tuning a chunked segment is longer than the smallest
    // wave_max and every chunk but its last covers chunk_vectors 16-byte
    // vectors, so: states <= min(nseg, total / min_wave_max); work items <=
    // nseg + total / min_chunk_elems.  Each array starts on a 256-byte
    // boundary.
    if (nseg >= (1ull << 31) || total_elems > (1ull << 50))
        return 0;
    const uint64_t min_wave = std::min(kWaveMaxDefault[0],
                                       std::min(kWaveMaxDefault[1], kWaveMaxDefault[2]));
    const uint64_t min_chunk = xsum::segmented_chunk_vectors() * 2;   // binary64
    const uint64_t states = std::min<uint64_t>(nseg, total_elems / min_wave);
    const uint64_t items = nseg + total_elems / min_chunk + 1;
    return (size_t)(oneshot_layout(nseg, items, nseg, states).total);
}

xsum_status_t xsum_exact_sum_segmented(const void *base, const xsum_segment_t *segs,
                                       uint64_t nseg, int out_dtype, void *out,
                                       uint32_t *flags, void *workspace, size_t ws_bytes,
                                       void *stream)
{
    if (nseg == 0)
        return XSUM_OK;
    if (segs == nullptr || base == nullptr || out == nullptr || workspace == nullptr)
        return api_fail(XSUM_EINVAL, "segs, base, out or workspace is NULL");
    if ((uintptr_t)base % 16 != 0)
        return api_fail(XSUM_EINVAL, "base must be 16-byte aligned");
    if ((uintptr_t)out % 8 != 0 || (uintptr_t)workspace % 256 != 0 ||
        (flags && (uintptr_t)flags % 4 != 0))
        return api_fail(XSUM_EINVAL, "misaligned out, flags or workspace (256 bytes)");
    if (nseg >= (1ull << 31))
        return api_fail(XSUM_ERANGE, "at most 2^31 - 1 segments");
    hipStream_t s = (hipStream_t)stream;
    int dev, cus;
    xsum_status_t st = xsum::api_current_cus(&dev, &cus);
    if (st != XSUM_OK)
        return st;
    // Work already queued on the stream may still produce the table or use
    // this workspace: wait for it before reading the one or writing the other.
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return api_hip_fail(e, "hipStreamSynchronize");
    std::vector<xsum_segment_t> table;
    const xsum_segment_t *host_segs = segs;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, segs) == hipSuccess &&
        attr.type == hipMemoryTypeDevice) {
        table.resize(nseg);
        e = hipMemcpy(table.data(), segs, nseg * sizeof(xsum_segment_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return api_hip_fail(e, "segment table download");
        host_segs = table.data();
    } else {
        (void)hipGetLastError();   // a host pointer: the query may leave an error
    }
    HostPlan hp;
    st = make_plan(host_segs, nseg, out_dtype, nullptr, cus, hp);
    if (st != XSUM_OK)
        return st;
    const OneshotLayout L = oneshot_layout(nseg, hp.tasks.size(), hp.lanes.size(), hp.nslots);
    if (ws_bytes < L.total)
        return api_fail(XSUM_EINVAL, "workspace smaller than this table needs (" +
                                         std::to_string(L.total) + " bytes)");
    uint8_t *ws = (uint8_t *)workspace;
    e = hipMemcpy(ws + L.segs, host_segs, nseg * sizeof(xsum::SegDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess && !hp.tasks.empty())
        e = hipMemcpy(ws + L.tasks, hp.tasks.data(), hp.tasks.size() * sizeof(xsum::SegTask),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !hp.lanes.empty())
        e = hipMemcpy(ws + L.lanes, hp.lanes.data(), hp.lanes.size() * sizeof(xsum::SegLane),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return api_hip_fail(e, "plan upload");
    // control words and chunk states start at zero
    e = xsum::launch_zero_words((uint64_t *)ws, L.segs / 8, s);
    if (e == hipSuccess)
        e = xsum::launch_segmented(base, (const xsum::SegDesc *)(ws + L.segs),
                                   (const xsum::SegTask *)(ws + L.tasks),
                                   (uint32_t)hp.tasks.size(),
                                   (const xsum::SegLane *)(ws + L.lanes),
                                   (xsum_acc_t *)(ws + xsum::kSegCtlBytes), (xsum::SegCtl *)ws,
                                   out_dtype, (uint64_t *)out, flags, hp.blocks, s);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_segmented_run(const xsum_plan_t *plan, const void *base,
                                 void *out, uint32_t *flags, void *workspace,
                                 size_t ws_bytes, void *stream)
{
    if (plan == nullptr)
        return api_fail(XSUM_EINVAL, "plan is NULL");
    if (plan->nseg == 0)
        return XSUM_OK;
    if (base == nullptr || out == nullptr || workspace == nullptr)
        return api_fail(XSUM_EINVAL, "base, out or workspace is NULL");
    if ((uintptr_t)base % 16 != 0)
        return api_fail(XSUM_EINVAL, "base must be 16-byte aligned");
    if ((uintptr_t)out % 8 != 0 || (uintptr_t)workspace % 8 != 0 ||
        (flags && (uintptr_t)flags % 4 != 0))
        return api_fail(XSUM_EINVAL, "misaligned out, flags or workspace");
    if (ws_bytes < plan->info.workspace_bytes)
        return api_fail(XSUM_EINVAL, "workspace smaller than xsum_plan_workspace_size()");
    int dev;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return api_hip_fail(e, "hipGetDevice");
    if (dev != plan->device)
        return api_fail(XSUM_EINVAL, "plan was built for another device");
    uint8_t *ws = (uint8_t *)workspace;
    e = xsum::launch_segmented(base, plan->d_segs, plan->d_tasks, plan->ntasks,
                               plan->d_lanes, (xsum_acc_t *)(ws + xsum::kSegCtlBytes),
                               (xsum::SegCtl *)ws, plan->out_mode, (uint64_t *)out,
                               flags, plan->blocks, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_segmented_run_noalloc(const xsum_plan_t *plan, const void *base,
                                         void *out, uint32_t *flags, void *stream)
{
    // the scratch array's device address, looked up once per device
    static std::mutex mu;
    static std::vector<void *> addr;
    if (plan == nullptr)
        return api_fail(XSUM_EINVAL, "plan is NULL");
    if (plan->info.workspace_bytes > kNoallocScratchBytes)
        return api_fail(XSUM_ERANGE, "plan needs " + std::to_string(plan->info.workspace_bytes) +
                                         " workspace bytes; the allocation-free run holds " +
                                         std::to_string(kNoallocScratchBytes) +
                                         " (at most 1820 chunked segments)");
    if (plan->nseg == 0)
        return XSUM_OK;
    int dev;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return api_hip_fail(e, "hipGetDevice");
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        if ((size_t)dev >= addr.size())
            addr.resize((size_t)dev + 1, nullptr);
        if (addr[dev] == nullptr) {
            void *ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return api_hip_fail(e, "hipGetSymbolAddress(scratch)");
            addr[dev] = ptr;
        }
        ws = addr[dev];
    }
    // a previous call may have stopped before its end: the control words and
    // chunk states this plan uses start at zero (a fill kernel, no memset, so
    // the call may be captured)
    e = xsum::launch_zero_words((uint64_t *)ws, (plan->info.workspace_bytes + 7) / 8,
                                (hipStream_t)stream);
    if (e != hipSuccess)
        return api_hip_fail(e, "kernel launch");
    return xsum_segmented_run(plan, base, out, flags, ws, kNoallocScratchBytes, stream);
}

xsum_status_t xsum_segmented_workspace_init(void *workspace, size_t ws_bytes,
                                            void *stream)
{
    if (ws_bytes == 0)
        return XSUM_OK;
    if (workspace == nullptr || (uintptr_t)workspace % 8 != 0 || ws_bytes % 8 != 0)
        return api_fail(XSUM_EINVAL, "workspace NULL, misaligned or not a multiple of 8 bytes");
    hipError_t e = xsum::launch_zero_words((uint64_t *)workspace, ws_bytes / 8,
                                           (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_segmented_capture(const xsum_plan_t *plan, const void *base,
                                     void *out, uint32_t *flags,
                                     void *workspace, size_t ws_bytes,
                                     void **graph_exec)
{
    if (graph_exec == nullptr)
        return api_fail(XSUM_EINVAL, "graph_exec is NULL");
    *graph_exec = nullptr;
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess)
        return api_hip_fail(e, "hipStreamCreate");
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return api_hip_fail(e, "hipStreamBeginCapture");
    }
    xsum_status_t st = xsum_segmented_run(plan, base, out, flags, workspace, ws_bytes, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (st != XSUM_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return api_hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return api_hip_fail(e, "hipGraphInstantiate");
    *graph_exec = (void *)ex;
    return XSUM_OK;
}

xsum_status_t xsum_graph_launch(void *graph_exec, void *stream)
{
    if (graph_exec == nullptr)
        return api_fail(XSUM_EINVAL, "graph_exec is NULL");
    hipError_t e = hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "hipGraphLaunch");
}

void xsum_graph_destroy(void *graph_exec)
{
    if (graph_exec)
        (void)hipGraphExecDestroy((hipGraphExec_t)graph_exec);
}

uint64_t xsum_batch_item_tasks(uint64_t ptr, uint64_t length, int dtype,
                               uint64_t chunk_vectors)
{
    if (dtype < 0 || dtype > 2 || chunk_vectors == 0)
        return 1;
    uint64_t head = ((16 - (ptr & 15)) & 15) / (uint64_t)kBytes[dtype];
    if (head > length)
        head = length;
    const uint64_t nvs = (length - head) / (uint64_t)kPerVec[dtype];
    const uint64_t nch = (nvs + chunk_vectors - 1) / chunk_vectors;
    return nch ? nch : 1;
}

xsum_status_t xsum_batch_add(const xsum_batch_item_t *items, uint32_t nitems,
                             uint64_t ntasks, uint64_t chunk_vectors,
                             xsum_acc_t *states, void *ctl, void *stream)
{
    if (nitems == 0 || ntasks == 0)
        return XSUM_OK;
    if (items == nullptr || states == nullptr || ctl == nullptr)
        return api_fail(XSUM_EINVAL, "items, states or ctl is NULL");
    if (ntasks >= (1ull << 32) - 65536)
        return api_fail(XSUM_ERANGE, "too many work items in one batch");
    if (chunk_vectors < 64 || chunk_vectors > (1ull << 26))
        return api_fail(XSUM_ERANGE, "chunk_vectors out of range [64, 2^26]");
    int dev, cus;
    xsum_status_t st = xsum::api_current_cus(&dev, &cus);
    if (st != XSUM_OK)
        return st;
    uint64_t blocks = 4ull * (uint64_t)cus;
    if (blocks > ntasks)
        blocks = ntasks;
    hipError_t e = xsum::launch_batch_add((const xsum::BatchItem *)items, nitems, ntasks,
                                          chunk_vectors, states, (xsum::SegCtl *)ctl,
                                          (int)blocks, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "kernel launch");
}

xsum_status_t xsum_batch_finalize(const uint32_t *slots, const uint32_t *fmts,
                                  uint32_t n, xsum_acc_t *states, void *out,
                                  uint32_t *flags, void *stream)
{
    if (n == 0)
        return XSUM_OK;
    if (slots == nullptr || fmts == nullptr || states == nullptr || out == nullptr)
        return api_fail(XSUM_EINVAL, "slots, fmts, states or out is NULL");
    hipError_t e = xsum::launch_batch_finalize(slots, fmts, n, states, (uint64_t *)out,
                                               flags, (hipStream_t)stream);
    return e == hipSuccess ? XSUM_OK : api_hip_fail(e, "kernel launch");
}

}  // extern "C"
