// Host-side declarations shared by the solver's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "rgb_device.hpp"

struct rgb_ctx;

namespace rgb {

constexpr int kClasses = 16;     // LP size classes: ceil(log2 m), capped
constexpr int kBinBlocks = 256;  // blocks of the binning passes
constexpr int kQueues = 8;       // device queue parts (one per XCD of an MI355X)
constexpr int kHeadStride = 32;  // ints between queue heads (one 128-byte line each)

// Queue description written by the scan pass: classes in queue order
// (largest first), their entry ranges in `order`, and the cumulative count
// of sub-batches (64/G LPs each).
struct QueueHeader {
    int num_sb;     // sub-batches in total
    int dyn_begin;  // first sub-batch handed out by the queue
    int pad[2];
    int e_start[kClasses];
    int e_end[kClasses];
    int sb_end[kClasses];
    int lg[kClasses];
};

// Device workspace of one solve in flight.
struct Workspace {
    QueueHeader* q;
    int32_t* heads;   // [kQueues * kHeadStride] queue heads, one cache line apart
    int32_t* blocks;  // [kBinBlocks * kClasses] per-block class counts, then queue offsets
    int32_t* order;   // [num_lps] queue: LP ids, largest class first
    uint8_t* cls;     // [num_lps] size class per LP
};

// log2(lanes per LP) for each size class; the share of sub-batches (in
// 1/1024) left to the dynamic queue; sub-batches per queue pop.
struct PersistPlan {
    int log2_lanes[kClasses];
    int dyn_frac_1024;
    int chunk;
};

// Device of a context (for the server, which only sees the opaque type).
int ctx_device(const struct ::rgb_ctx* ctx);

// State of rgb_solve_batch_host (streams, device and pinned chunk buffers),
// kept in the context and freed with it.
struct HostPath;
HostPath*& ctx_host_path(struct ::rgb_ctx* ctx);
void destroy_host_path(HostPath* h);

hipError_t launch_persistent(const Problem& P, const Workspace& W, const PersistPlan& plan, int grid, bool binned,
                             hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end);
int persist_blocks_per_cu();
hipError_t launch_plain(const Problem& P, hipStream_t stream);
hipError_t launch_group(const Problem& P, int lanes_per_lp, hipStream_t stream);
bool group_supported(int lanes_per_lp);
hipError_t launch_pool(const Problem& P, int lanes_per_lp, int rows_per_lane, int wait8, hipStream_t stream);
bool pool_supported(int lanes_per_lp, int rows_per_lane);

}  // namespace rgb
