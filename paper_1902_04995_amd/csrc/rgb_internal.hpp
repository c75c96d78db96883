// Host-side declarations shared by the solver's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>

#include "rgb_device.hpp"

struct rgb_ctx;

namespace rgb {

constexpr int kClasses = 16;     // LP size classes: ceil(log2 m), capped
constexpr int kBinBlocks = 256;  // blocks of the binning passes
constexpr int kQueues = 8;       // device queue parts (one per XCD of an MI355X)
constexpr int kHeadStride = 32;  // ints between queue heads (one 128-byte line each)
// log2_lanes value of a size class whose LPs are each solved by one whole
// workgroup with its rows staged in LDS (the wide kernel), not by a group of
// 4..64 lanes.
constexpr int kWideLg = 8;

// Queue description written by the scan pass: classes in queue order (the
// wide classes first, then the others, each part largest first), their entry
// ranges in `order`, and the cumulative count of sub-batches (64/G LPs each;
// a wide class has none: its LPs are entries [0, n_wide) of the queue, taken
// by the wide kernel through wide_head).
struct QueueHeader {
    int num_sb;     // sub-batches in total
    int dyn_begin;  // first sub-batch handed out by the queue
    int n_wide;     // LPs of the wide classes
    int wide_head;  // next of them to take (reset by the scan pass)
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

// One device's entry of a persisted tuning table (rgb_table.cpp): the
// family and its scalar knobs, and lanes per LP for the size classes that
// were tuned.
struct TableEntry {
    int variant = 3;
    int log2_lanes[kClasses] = {};
    bool tuned[kClasses] = {};
    int batched_lanes = 16, queue_share = 128, chunk = 1, grid = 0;
    int pool_lanes = 4, pool_wait = 2, pool_rows = 4;
    double ms = 0.0;
};
// 1: entry found and applied to `out` (fields not in the file keep their
// values), 0: no entry for the device (or no file), -1: unreadable table.
int table_load(const char* path, const std::string& device_key, TableEntry& out);
// Merge `e` into the table at `path` (created if missing); 0 or -1.
int table_save(const char* path, const std::string& device_key, const TableEntry& e);

// Device of a context (for the server, which only sees the opaque type).
int ctx_device(const struct ::rgb_ctx* ctx);
// Give the context's workspace for solves on `stream` room for num_lps LPs
// now (a later larger solve on that stream would otherwise reallocate it,
// synchronising the stream).  False on failure.
bool reserve_workspace(struct ::rgb_ctx* ctx, void* stream, int64_t num_lps);

// Copy `bytes` bytes with a kernel on `stream` (not a DMA-engine copy), so
// that the copy, the kernels around it and a completion event recorded after
// it sit in one in-order queue.  Either side may be host memory given by its
// device-visible address.  Returns false if the launch fails.
bool launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

// State of rgb_solve_batch_host (streams, device and pinned chunk buffers),
// kept in the context and freed with it.
struct HostPath;
HostPath*& ctx_host_path(struct ::rgb_ctx* ctx);
void destroy_host_path(HostPath* h);

// The binned or persistent solve: binning, queue set-up, the wide kernel
// (wide_grid workgroups) when a class is wide, then the group kernel.
hipError_t launch_persistent(const Problem& P, const Workspace& W, const PersistPlan& plan, int grid, int wide_grid,
                             bool binned, hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end);
int persist_blocks_per_cu();
int wide_blocks_per_cu();
hipError_t launch_plain(const Problem& P, hipStream_t stream);
// The FP64 fix-up of LPs a fast kernel deferred; enqueued after every solve.
hipError_t launch_fixup(const Problem& P, hipStream_t stream);
hipError_t launch_group(const Problem& P, int lanes_per_lp, hipStream_t stream);
bool group_supported(int lanes_per_lp);
hipError_t launch_pool(const Problem& P, int lanes_per_lp, int rows_per_lane, int wait8, hipStream_t stream);
bool pool_supported(int lanes_per_lp, int rows_per_lane);

}  // namespace rgb
