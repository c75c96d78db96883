// C ABI of the batched 2D LP solver: argument checks, contexts, dispatch,
// autotuning and captured plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rgb.h"
#include "rgb_internal.hpp"

namespace {

// Device workspace of the solves issued on one stream (solves on one stream
// run in order, so they can share it), or of one plan.
struct WsSlot {
    void* stream = nullptr;
    void* mem = nullptr;
    int64_t cap = 0;
    rgb::Workspace ws{};
};

constexpr int kMaxStreams = 32;

// Workspace of rgb_solve_batch_noalloc: the binning and queue state of one
// solve of at most kScratchMaxLps LPs, laid out as grow_workspace lays out an
// allocated one (queue header and heads, per-block class counts, the queue of
// LP ids, the class per LP).  Every field is written by the binning kernels
// of the solve that uses it, so nothing needs clearing between calls.
constexpr int64_t kScratchMaxLps = int64_t(1) << 20;
constexpr size_t kScratchBlocksAt = 2048;
constexpr size_t kScratchOrderAt = kScratchBlocksAt + (size_t)rgb::kBinBlocks * rgb::kClasses * 4;
constexpr size_t kScratchClsAt = kScratchOrderAt + (size_t)kScratchMaxLps * 4;
constexpr size_t kScratchBytes = kScratchClsAt + (size_t)kScratchMaxLps;
static_assert(kScratchOrderAt % 256 == 0 && kScratchClsAt % 256 == 0, "scratch layout");

}  // namespace

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it takes the device's address from
// hipGetSymbolAddress (scratch_address below) and passes that to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct rgb_ctx {
    int device = 0;
    std::string device_key;  // "<name> <arch> <CUs>cu": the tuning table's key
    int num_cus = 0;
    int persist_blocks_per_cu = 1;
    int wide_blocks_per_cu = 1;
    rgb_tuning_t tuning{};
    std::vector<WsSlot> slots;
    rgb::HostPath* host = nullptr;  // rgb_solve_batch_host state, made on first use
    void* scratch = nullptr;        // this device's address of `scratch` (null: lookup failed)
    std::string last_error;
};

struct rgb_plan {
    rgb_ctx_t* ctx = nullptr;
    WsSlot ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

rgb_err_t fail(rgb_ctx_t* ctx, rgb_err_t code, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

// Makes a device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = prev == dev || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

bool lanes_ok(int g) { return g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

// Lanes per LP by size class before any tuning.
void default_tuning(rgb_tuning_t& t) {
    std::memset(&t, 0, sizeof(t));
    t.variant = RGB_VARIANT_BINNED;
    for (int c = 0; c < rgb::kClasses; ++c) {
        int lg = 6;
        if (c <= 4) lg = 2;
        else if (c <= 6) lg = 3;
        else if (c <= 8) lg = 4;
        else if (c <= 9) lg = 5;
        t.log2_lanes[c] = lg;
    }
    t.batched_lanes = 16;
    t.queue_share = 128;
    t.chunk = 1;
    t.grid = 0;
    t.pool_lanes = 4;
    t.pool_wait = 2;
    t.pool_rows = 4;
}

bool tuning_valid(const rgb_tuning_t& t) {
    if (t.variant != RGB_VARIANT_PERSISTENT && t.variant != RGB_VARIANT_BINNED && t.variant != RGB_VARIANT_BATCHED &&
        t.variant != RGB_VARIANT_POOLED)
        return false;
    for (int c = 0; c < rgb::kClasses; ++c)
        if ((t.log2_lanes[c] < 2 || t.log2_lanes[c] > 6) && t.log2_lanes[c] != rgb::kWideLg) return false;
    return lanes_ok(t.batched_lanes) && t.queue_share >= 0 && t.queue_share <= 1024 && t.chunk >= 1 &&
           t.grid >= 0 && rgb::pool_supported(t.pool_lanes, t.pool_rows) && t.pool_wait >= 0 && t.pool_wait <= 8;
}

rgb::TableEntry table_entry_of(const rgb_tuning_t& t) {
    rgb::TableEntry e;
    e.variant = t.variant;
    for (int c = 0; c < rgb::kClasses; ++c) e.log2_lanes[c] = t.log2_lanes[c];
    e.batched_lanes = t.batched_lanes;
    e.queue_share = t.queue_share;
    e.chunk = t.chunk;
    e.grid = t.grid;
    e.pool_lanes = t.pool_lanes;
    e.pool_wait = t.pool_wait;
    e.pool_rows = t.pool_rows;
    e.ms = t.ms;
    return e;
}

rgb_tuning_t tuning_of(const rgb::TableEntry& e) {
    rgb_tuning_t t;
    std::memset(&t, 0, sizeof(t));
    t.variant = e.variant;
    for (int c = 0; c < rgb::kClasses; ++c) t.log2_lanes[c] = e.log2_lanes[c];
    t.batched_lanes = e.batched_lanes;
    t.queue_share = e.queue_share;
    t.chunk = e.chunk;
    t.grid = e.grid;
    t.pool_lanes = e.pool_lanes;
    t.pool_wait = e.pool_wait;
    t.pool_rows = e.pool_rows;
    t.ms = (float)e.ms;
    return t;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// (Re)allocate a workspace for num_lps LPs.  Never during capture.
rgb_err_t grow_workspace(rgb_ctx_t* ctx, WsSlot& slot, int64_t num_lps) {
    if (slot.mem && slot.cap >= num_lps) return RGB_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (slot.stream && hipStreamIsCapturing(reinterpret_cast<hipStream_t>(slot.stream), &cs) == hipSuccess &&
        cs != hipStreamCaptureStatusNone)
        return fail(ctx, RGB_ERR_INVALID_ARG, "workspace must grow but the stream is being captured");
    static_assert(sizeof(rgb::QueueHeader) <= 1024, "queue header");
    static_assert(rgb::kQueues * rgb::kHeadStride * 4 <= 1024, "queue heads");
    int64_t cap = num_lps < 1024 ? 1024 : num_lps + num_lps / 4;
    size_t head_bytes = 2048;
    size_t blocks_off = head_bytes;
    size_t order_off = blocks_off + (size_t)rgb::kBinBlocks * rgb::kClasses * 4;
    size_t cls_off = align_up(order_off + (size_t)cap * 4, 256);
    size_t total = cls_off + align_up((size_t)cap, 256);
    if (slot.mem) {
        if (slot.stream) (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(slot.stream));
        else (void)hipDeviceSynchronize();
        (void)hipFree(slot.mem);
        slot.mem = nullptr;
        slot.cap = 0;
    }
    // No clearing: the binning kernels of every solve write each field before
    // any kernel reads it.  A host-side clear would also be unordered with
    // the caller's stream: a hipMemset goes to the null stream, which a
    // non-blocking stream does not wait for, so it could land after this
    // solve's queue set-up and empty the queue.
    void* mem = nullptr;
    if (hipMalloc(&mem, total) != hipSuccess) return fail(ctx, RGB_ERR_OOM, "workspace of %zu bytes", total);
    char* base = static_cast<char*>(mem);
    slot.mem = mem;
    slot.cap = cap;
    slot.ws.q = reinterpret_cast<rgb::QueueHeader*>(base);
    slot.ws.heads = reinterpret_cast<int32_t*>(base + 1024);
    slot.ws.blocks = reinterpret_cast<int32_t*>(base + blocks_off);
    slot.ws.order = reinterpret_cast<int32_t*>(base + order_off);
    slot.ws.cls = reinterpret_cast<uint8_t*>(base + cls_off);
    return RGB_OK;
}

// Device address of `scratch` on the current device `dev`, looked up once per
// device (each device holds its own copy at its own address); null if the
// lookup fails.
void* scratch_address(int dev) {
    static std::mutex mu;
    static std::vector<std::pair<int, void*>> known;
    std::lock_guard<std::mutex> lk(mu);
    for (const auto& k : known)
        if (k.first == dev) return k.second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();  // clear the error so later calls do not report it
        return nullptr;
    }
    known.emplace_back(dev, p);
    return p;
}

// The workspace of rgb_solve_batch_noalloc inside the device's `scratch`.
rgb::Workspace scratch_workspace(void* base_ptr) {
    char* base = static_cast<char*>(base_ptr);
    rgb::Workspace w{};
    w.q = reinterpret_cast<rgb::QueueHeader*>(base);
    w.heads = reinterpret_cast<int32_t*>(base + 1024);
    w.blocks = reinterpret_cast<int32_t*>(base + kScratchBlocksAt);
    w.order = reinterpret_cast<int32_t*>(base + kScratchOrderAt);
    w.cls = reinterpret_cast<uint8_t*>(base + kScratchClsAt);
    return w;
}

// Workspace of the solves issued on `stream`.
rgb_err_t stream_workspace(rgb_ctx_t* ctx, void* stream, int64_t num_lps, rgb::Workspace& out) {
    WsSlot* slot = nullptr;
    for (auto& s : ctx->slots)
        if (s.stream == stream) slot = &s;
    if (!slot) {
        if ((int)ctx->slots.size() >= kMaxStreams)
            return fail(ctx, RGB_ERR_BUSY, "more than %d streams used with one context", kMaxStreams);
        ctx->slots.push_back(WsSlot{});
        slot = &ctx->slots.back();
        slot->stream = stream;
    }
    rgb_err_t rc = grow_workspace(ctx, *slot, num_lps);
    if (rc != RGB_OK) return rc;
    out = slot->ws;
    return RGB_OK;
}

struct Batch {
    int64_t num_lps, num_constraints;
    const int64_t* offsets;
    const float *ax, *ay, *b, *cx, *cy;
    float *x_out, *y_out;
    int32_t* status_out;
};

rgb_err_t check_batch(rgb_ctx_t* ctx, const Batch& B) {
    if (B.num_lps < 0 || B.num_constraints < 0)
        return fail(ctx, RGB_ERR_INVALID_ARG, "negative num_lps (%lld) or num_constraints (%lld)",
                    (long long)B.num_lps, (long long)B.num_constraints);
    if (B.num_lps == 0) return RGB_OK;
    if (!B.offsets || !B.cx || !B.cy || !B.x_out || !B.y_out || !B.status_out)
        return fail(ctx, RGB_ERR_INVALID_ARG, "null per-LP pointer");
    if (B.num_constraints > 0 && (!B.ax || !B.ay || !B.b)) return fail(ctx, RGB_ERR_INVALID_ARG, "null row pointer");
    if (B.num_lps > (int64_t)0x7fffffff - rgb::kClasses)
        return fail(ctx, RGB_ERR_TOO_LARGE, "num_lps above 2^31 - 17");
    return RGB_OK;
}

rgb::Problem make_problem(const Batch& B, int32_t* n1d) {
    rgb::Problem P{};
    P.offsets = B.offsets;
    P.ax = B.ax;
    P.ay = B.ay;
    P.b = B.b;
    P.cx = B.cx;
    P.cy = B.cy;
    P.x_out = B.x_out;
    P.y_out = B.y_out;
    P.status = B.status_out;
    P.n1d = n1d;
    P.order = nullptr;
    P.num_lps = B.num_lps;
    P.num_constraints = B.num_constraints;
    return P;
}

// Effective configuration of a call: ctx's tuning with the opts overrides.
rgb_err_t resolve(rgb_ctx_t* ctx, const rgb_solve_opts_t& o, int& variant, rgb_tuning_t& cfg) {
    cfg = ctx->tuning;
    variant = o.variant;
    if (variant < RGB_VARIANT_AUTO || variant > RGB_VARIANT_POOLED)
        return fail(ctx, RGB_ERR_INVALID_ARG, "unknown variant %d", variant);
    if (variant == RGB_VARIANT_AUTO) variant = cfg.variant;
    if (o.lanes_per_lp) {
        if (!lanes_ok(o.lanes_per_lp))
            return fail(ctx, RGB_ERR_INVALID_ARG, "lanes_per_lp=%d is not one of 4, 8, 16, 32, 64", o.lanes_per_lp);
        if (variant == RGB_VARIANT_POOLED && !rgb::pool_supported(o.lanes_per_lp, 1))
            return fail(ctx, RGB_ERR_INVALID_ARG, "POOLED takes 4, 8 or 16 lanes per LP, not %d", o.lanes_per_lp);
        cfg.batched_lanes = o.lanes_per_lp;
        for (int c = 0; c < rgb::kClasses; ++c) cfg.log2_lanes[c] = __builtin_ctz(o.lanes_per_lp);
        if (rgb::pool_supported(o.lanes_per_lp, 1)) cfg.pool_lanes = o.lanes_per_lp;
    }
    if (o.pool_wait < -1 || o.pool_wait > 8)
        return fail(ctx, RGB_ERR_INVALID_ARG, "pool_wait %d outside [-1, 8]", o.pool_wait);
    if (o.pool_wait) cfg.pool_wait = o.pool_wait < 0 ? 0 : o.pool_wait;
    if (o.pool_rows && !rgb::pool_supported(4, o.pool_rows))
        return fail(ctx, RGB_ERR_INVALID_ARG, "pool_rows %d is not one of 1, 2, 4", o.pool_rows);
    if (o.pool_rows) cfg.pool_rows = o.pool_rows;
    if (o.chunk < 0 || o.grid < 0) return fail(ctx, RGB_ERR_INVALID_ARG, "negative chunk or grid");
    if (o.chunk) cfg.chunk = o.chunk;
    if (o.grid) cfg.grid = o.grid;
    if (o.queue_share < -1 || o.queue_share > 1024)
        return fail(ctx, RGB_ERR_INVALID_ARG, "queue_share %d outside [-1, 1024]", o.queue_share);
    if (o.queue_share) cfg.queue_share = o.queue_share < 0 ? 0 : o.queue_share;
    return RGB_OK;
}

// Enqueue one solve.  W is needed by PERSISTENT and BINNED only.
rgb_err_t enqueue(rgb_ctx_t* ctx, const rgb::Problem& P, int variant, const rgb_tuning_t& cfg,
                  const rgb::Workspace* W, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e;
    // every family is followed by the FP64 fix-up of the LPs it deferred;
    // the events bracket both
    if (variant == RGB_VARIANT_PLAIN) {
        if (ev0) (void)hipEventRecord(ev0, st);
        e = rgb::launch_plain(P, st);
        if (e == hipSuccess) e = rgb::launch_fixup(P, st);
        if (ev1) (void)hipEventRecord(ev1, st);
    } else if (variant == RGB_VARIANT_BATCHED) {
        if (ev0) (void)hipEventRecord(ev0, st);
        e = rgb::launch_group(P, cfg.batched_lanes, st);
        if (e == hipSuccess) e = rgb::launch_fixup(P, st);
        if (ev1) (void)hipEventRecord(ev1, st);
    } else if (variant == RGB_VARIANT_POOLED) {
        if (ev0) (void)hipEventRecord(ev0, st);
        e = rgb::launch_pool(P, cfg.pool_lanes, cfg.pool_rows, cfg.pool_wait, st);
        if (e == hipSuccess) e = rgb::launch_fixup(P, st);
        if (ev1) (void)hipEventRecord(ev1, st);
    } else {
        rgb::PersistPlan plan{};
        for (int c = 0; c < rgb::kClasses; ++c) plan.log2_lanes[c] = cfg.log2_lanes[c];
        plan.dyn_frac_1024 = cfg.queue_share;
        plan.chunk = cfg.chunk;
        int grid = cfg.grid ? cfg.grid : ctx->num_cus * ctx->persist_blocks_per_cu;
        e = rgb::launch_persistent(P, *W, plan, grid, ctx->num_cus * ctx->wide_blocks_per_cu,
                                   variant == RGB_VARIANT_BINNED, st, ev0, ev1);
    }
    if (e != hipSuccess) return fail(ctx, RGB_ERR_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return RGB_OK;
}

}  // namespace

int rgb::ctx_device(const rgb_ctx* ctx) { return ctx->device; }
bool rgb::reserve_workspace(rgb_ctx* ctx, void* stream, int64_t num_lps) {
    rgb::Workspace w;
    return stream_workspace(ctx, stream, num_lps, w) == RGB_OK;
}
rgb::HostPath*& rgb::ctx_host_path(rgb_ctx* ctx) { return ctx->host; }

extern "C" {

const char* rgb_version(void) { return "rgb-mi355x 0.2 (gfx950)"; }

rgb_err_t rgb_ctx_create(int device, const rgb_ctx_opts_t* opts, rgb_ctx_t** out) {
    if (!out) return RGB_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return RGB_ERR_DEVICE;
    if (device < 0 || device >= n) return RGB_ERR_INVALID_ARG;
    rgb_ctx_t* ctx = new (std::nothrow) rgb_ctx_t();
    if (!ctx) return RGB_ERR_OOM;
    ctx->device = device;
    DeviceGuard guard(device);
    hipDeviceProp_t prop;
    if (!guard.ok || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return RGB_ERR_DEVICE;
    }
    ctx->num_cus = prop.multiProcessorCount;
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    ctx->device_key = std::string(prop.name) + " " + arch + " " + std::to_string(prop.multiProcessorCount) + "cu";
    ctx->persist_blocks_per_cu = rgb::persist_blocks_per_cu();
    ctx->wide_blocks_per_cu = rgb::wide_blocks_per_cu();
    ctx->scratch = scratch_address(device);
    default_tuning(ctx->tuning);
    if (opts && opts->tuning_table) {
        rgb::TableEntry e = table_entry_of(ctx->tuning);
        const int r = rgb::table_load(opts->tuning_table, ctx->device_key, e);
        rgb_tuning_t t = tuning_of(e);
        if (r < 0 || (r == 1 && !tuning_valid(t))) {
            delete ctx;
            return RGB_ERR_INVALID_ARG;
        }
        if (r == 1) ctx->tuning = t;
    }
    *out = ctx;
    return RGB_OK;
}

rgb_err_t rgb_ctx_destroy(rgb_ctx_t* ctx) {
    if (!ctx) return RGB_OK;
    {
        DeviceGuard guard(ctx->device);
        rgb::destroy_host_path(ctx->host);
        for (auto& s : ctx->slots)
            if (s.mem) (void)hipFree(s.mem);
    }
    delete ctx;
    return RGB_OK;
}

const char* rgb_ctx_last_error(const rgb_ctx_t* ctx) {
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

rgb_err_t rgb_ctx_get_tuning(const rgb_ctx_t* ctx, rgb_tuning_t* out) {
    if (!ctx || !out) return RGB_ERR_INVALID_ARG;
    *out = ctx->tuning;
    return RGB_OK;
}

rgb_err_t rgb_ctx_set_tuning(rgb_ctx_t* ctx, const rgb_tuning_t* tuning) {
    if (!ctx || !tuning) return RGB_ERR_INVALID_ARG;
    if (!tuning_valid(*tuning)) return fail(ctx, RGB_ERR_INVALID_ARG, "invalid tuning");
    ctx->tuning = *tuning;
    return RGB_OK;
}

rgb_err_t rgb_solve_batch(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                          const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                          float* x_out, float* y_out, int32_t* status_out, const rgb_solve_opts_t* opts,
                          void* stream) {
    if (!ctx) return RGB_ERR_INVALID_ARG;
    ctx->last_error.clear();
    Batch B{num_lps, num_constraints, offsets, ax, ay, b, cx, cy, x_out, y_out, status_out};
    rgb_err_t rc = check_batch(ctx, B);
    if (rc != RGB_OK || num_lps == 0) return rc;
    rgb_solve_opts_t o{};
    if (opts) o = *opts;
    int variant;
    rgb_tuning_t cfg;
    if ((rc = resolve(ctx, o, variant, cfg)) != RGB_OK) return rc;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, RGB_ERR_DEVICE, "cannot select device %d", ctx->device);
    rgb::Workspace W{};
    if (variant == RGB_VARIANT_PERSISTENT || variant == RGB_VARIANT_BINNED)
        if ((rc = stream_workspace(ctx, stream, num_lps, W)) != RGB_OK) return rc;
    return enqueue(ctx, make_problem(B, o.n_1dlp_out), variant, cfg, &W, reinterpret_cast<hipStream_t>(stream),
                   reinterpret_cast<hipEvent_t>(o.ev_begin), reinterpret_cast<hipEvent_t>(o.ev_end));
}

rgb_err_t rgb_solve_batch_noalloc(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                                  const float* ax, const float* ay, const float* b, const float* cx,
                                  const float* cy, float* x_out, float* y_out, int32_t* status_out,
                                  const rgb_solve_opts_t* opts, void* stream) {
    if (!ctx) return RGB_ERR_INVALID_ARG;
    ctx->last_error.clear();
    Batch B{num_lps, num_constraints, offsets, ax, ay, b, cx, cy, x_out, y_out, status_out};
    rgb_err_t rc = check_batch(ctx, B);
    if (rc != RGB_OK || num_lps == 0) return rc;
    if (num_lps > kScratchMaxLps)
        return fail(ctx, RGB_ERR_TOO_LARGE, "rgb_solve_batch_noalloc takes at most %lld LPs, got %lld",
                    (long long)kScratchMaxLps, (long long)num_lps);
    rgb_solve_opts_t o{};
    if (opts) o = *opts;
    int variant;
    rgb_tuning_t cfg;
    if ((rc = resolve(ctx, o, variant, cfg)) != RGB_OK) return rc;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, RGB_ERR_DEVICE, "cannot select device %d", ctx->device);
    rgb::Workspace W{};
    if (variant == RGB_VARIANT_PERSISTENT || variant == RGB_VARIANT_BINNED) {
        if (!ctx->scratch) return fail(ctx, RGB_ERR_DEVICE, "no address for the static workspace on device %d",
                                       ctx->device);
        W = scratch_workspace(ctx->scratch);
    }
    return enqueue(ctx, make_problem(B, o.n_1dlp_out), variant, cfg, &W, reinterpret_cast<hipStream_t>(stream),
                   reinterpret_cast<hipEvent_t>(o.ev_begin), reinterpret_cast<hipEvent_t>(o.ev_end));
}

rgb_err_t rgb_autotune(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                       const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                       float* x_out, float* y_out, int32_t* status_out, int32_t reps, double budget_ms,
                       const char* table_path, void* stream, rgb_tuning_t* best) {
    if (!ctx) return RGB_ERR_INVALID_ARG;
    ctx->last_error.clear();
    Batch B{num_lps, num_constraints, offsets, ax, ay, b, cx, cy, x_out, y_out, status_out};
    rgb_err_t rc = check_batch(ctx, B);
    if (rc != RGB_OK) return rc;
    if (reps < 1 || reps > 1000) return fail(ctx, RGB_ERR_INVALID_ARG, "reps %d outside [1, 1000]", reps);
    if (num_lps == 0) {
        if (best) *best = ctx->tuning;
        return RGB_OK;
    }
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, RGB_ERR_DEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rgb::Workspace W{};
    if ((rc = stream_workspace(ctx, stream, num_lps, W)) != RGB_OK) return rc;
    const rgb::Problem P = make_problem(B, nullptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(ctx, RGB_ERR_DEVICE, "event create failed");
    }
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed_ms = [&] {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    };
    // median time of `reps` whole solves (binning included) with cfg
    auto measure = [&](const rgb_tuning_t& cfg, float& ms) -> rgb_err_t {
        std::vector<float> t;
        rgb_err_t r = enqueue(ctx, P, cfg.variant, cfg, &W, st, nullptr, nullptr);  // warm-up
        if (r != RGB_OK) return r;
        for (int i = 0; i < reps; ++i) {
            (void)hipEventRecord(e0, st);
            if ((r = enqueue(ctx, P, cfg.variant, cfg, &W, st, nullptr, nullptr)) != RGB_OK) return r;
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(ctx, RGB_ERR_DEVICE, "solve failed");
            float v = 0.0f;
            (void)hipEventElapsedTime(&v, e0, e1);
            t.push_back(v);
        }
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return RGB_OK;
    };
    rgb_tuning_t win = ctx->tuning;
    win.ms = 1e30f;
    // best of the class-aware families (persistent, binned) and the classes whose lanes were measured
    rgb_tuning_t class_best = ctx->tuning;
    bool class_tuned[rgb::kClasses] = {};
    auto try_cfg = [&](rgb_tuning_t cand) -> rgb_err_t {
        float ms = 0.0f;
        rgb_err_t r = measure(cand, ms);
        if (r != RGB_OK) return r;
        cand.ms = ms;
        if (ms < win.ms) win = cand;
        return RGB_OK;
    };
    auto tune = [&]() -> rgb_err_t {
        const rgb_tuning_t cur = ctx->tuning;
        rgb_err_t r;
        // 1. the kernel families with their default shapes, BATCHED at every width
        for (int v : {RGB_VARIANT_PERSISTENT, RGB_VARIANT_BINNED}) {
            rgb_tuning_t c = cur;
            c.variant = v;
            if ((r = try_cfg(c)) != RGB_OK) return r;
        }
        for (int g : {8, 16, 32, 64}) {
            rgb_tuning_t c = cur;
            c.variant = RGB_VARIANT_BATCHED;
            c.batched_lanes = g;
            if ((r = try_cfg(c)) != RGB_OK) return r;
        }
        // POOLED: scan width, rows per lane and wait threshold
        static const int kPool[][3] = {{4, 4, 2}, {4, 4, 0}, {4, 2, 2}, {8, 4, 2}, {8, 2, 2}, {8, 2, 0}, {16, 2, 2}};
        for (const auto& pc : kPool) {
            rgb_tuning_t c = cur;
            c.variant = RGB_VARIANT_POOLED;
            c.pool_lanes = pc[0];
            c.pool_rows = pc[1];
            c.pool_wait = pc[2];
            if ((r = try_cfg(c)) != RGB_OK) return r;
        }
        // 2. rows per size class, from a binning pass
        std::vector<uint8_t> cls((size_t)num_lps);
        std::vector<int64_t> offs((size_t)num_lps + 1);
        {
            rgb_tuning_t c = cur;
            c.variant = RGB_VARIANT_BINNED;
            if ((r = enqueue(ctx, P, c.variant, c, &W, st, nullptr, nullptr)) != RGB_OK) return r;
        }
        if (hipStreamSynchronize(st) != hipSuccess ||
            hipMemcpy(cls.data(), W.cls, (size_t)num_lps, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(offs.data(), offsets, offs.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(ctx, RGB_ERR_DEVICE, "reading the size classes failed");
        int64_t rows[rgb::kClasses] = {0}, total = 0;
        for (int64_t k = 0; k < num_lps; ++k) {
            int64_t m = offs[k + 1] - offs[k];
            if (m < 0) m = 0;
            rows[cls[k] & (rgb::kClasses - 1)] += m;
            total += m;
        }
        // 3. lanes per LP, class by class (largest share of rows first), for both binned families
        std::vector<int> order;
        for (int c = 0; c < rgb::kClasses; ++c)
            if (total > 0 && rows[c] * 25 >= total) order.push_back(c);
        std::sort(order.begin(), order.end(), [&](int a, int bb) { return rows[a] > rows[bb]; });
        rgb_tuning_t base = win;
        if (base.variant == RGB_VARIANT_BATCHED || base.variant == RGB_VARIANT_POOLED) {
            base = cur;
            base.variant = RGB_VARIANT_PERSISTENT;
        }
        for (int c : order) {
            if (elapsed_ms() > budget_ms) break;
            float best_ms = 1e30f;
            for (int v : {RGB_VARIANT_PERSISTENT, RGB_VARIANT_BINNED})
                for (int lg : {2, 3, 4, 5, 6, rgb::kWideLg}) {
                    rgb_tuning_t cand = base;
                    cand.variant = v;
                    cand.log2_lanes[c] = lg;
                    float ms = 0.0f;
                    if ((r = measure(cand, ms)) != RGB_OK) return r;
                    cand.ms = ms;
                    if (ms < win.ms) win = cand;
                    if (ms < best_ms) {
                        best_ms = ms;
                        class_best = cand;
                    }
                }
            class_tuned[c] = true;
            base = class_best;
        }
        // 4. queue share and chunk of the persistent kernel
        for (int share : {0, 128, 512, 1024})
            for (int chunk : {1, 2, 4}) {
                if (elapsed_ms() > budget_ms) return RGB_OK;
                if (share == 0 && chunk > 1) continue;
                rgb_tuning_t cand = base;
                cand.variant = RGB_VARIANT_PERSISTENT;
                cand.queue_share = share;
                cand.chunk = chunk;
                if ((r = try_cfg(cand)) != RGB_OK) return r;
            }
        return RGB_OK;
    };
    rc = tune();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != RGB_OK) return rc;
    ctx->tuning = win;
    if (best) *best = win;
    if (table_path) {
        // the family and knobs of the winner; lanes per class from the best
        // class-aware configuration, for the classes that were measured
        rgb::TableEntry e = table_entry_of(win);
        for (int c = 0; c < rgb::kClasses; ++c) {
            e.log2_lanes[c] = class_best.log2_lanes[c];
            e.tuned[c] = class_tuned[c];
        }
        if (rgb::table_save(table_path, ctx->device_key, e) != 0)
            return fail(ctx, RGB_ERR_INVALID_ARG, "cannot write the tuning table %s", table_path);
    }
    return RGB_OK;
}

rgb_err_t rgb_plan_create(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                          const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                          float* x_out, float* y_out, int32_t* status_out, const rgb_solve_opts_t* opts,
                          rgb_plan_t** out) {
    if (!ctx || !out) return RGB_ERR_INVALID_ARG;
    *out = nullptr;
    ctx->last_error.clear();
    Batch B{num_lps, num_constraints, offsets, ax, ay, b, cx, cy, x_out, y_out, status_out};
    rgb_err_t rc = check_batch(ctx, B);
    if (rc != RGB_OK) return rc;
    rgb_solve_opts_t o{};
    if (opts) o = *opts;
    int variant;
    rgb_tuning_t cfg;
    if ((rc = resolve(ctx, o, variant, cfg)) != RGB_OK) return rc;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, RGB_ERR_DEVICE, "cannot select device %d", ctx->device);
    rgb_plan_t* plan = new (std::nothrow) rgb_plan_t();
    if (!plan) return fail(ctx, RGB_ERR_OOM, "plan");
    plan->ctx = ctx;
    if ((rc = grow_workspace(ctx, plan->ws, num_lps)) != RGB_OK) {
        delete plan;
        return rc;
    }
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        rgb_plan_destroy(plan);
        return fail(ctx, RGB_ERR_DEVICE, "stream create failed");
    }
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (num_lps > 0)
            rc = enqueue(ctx, make_problem(B, o.n_1dlp_out), variant, cfg, &plan->ws.ws, cap,
                         reinterpret_cast<hipEvent_t>(o.ev_begin), reinterpret_cast<hipEvent_t>(o.ev_end));
        e = hipStreamEndCapture(cap, &plan->graph);
    }
    (void)hipStreamDestroy(cap);
    if (rc != RGB_OK || e != hipSuccess) {
        rgb_plan_destroy(plan);
        return rc != RGB_OK ? rc : fail(ctx, RGB_ERR_DEVICE, "capture failed: %s", hipGetErrorString(e));
    }
    if ((e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0)) != hipSuccess) {
        rgb_plan_destroy(plan);
        return fail(ctx, RGB_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    *out = plan;
    return RGB_OK;
}

rgb_err_t rgb_plan_launch(rgb_plan_t* plan, void* stream) {
    if (!plan || !plan->exec) return RGB_ERR_INVALID_ARG;
    DeviceGuard guard(plan->ctx->device);
    hipError_t e = hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(plan->ctx, RGB_ERR_DEVICE, "graph launch failed: %s", hipGetErrorString(e));
    return RGB_OK;
}

rgb_err_t rgb_plan_destroy(rgb_plan_t* plan) {
    if (!plan) return RGB_OK;
    DeviceGuard guard(plan->ctx->device);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->ws.mem) (void)hipFree(plan->ws.mem);
    delete plan;
    return RGB_OK;
}

}  // extern "C"
