// C ABI of the batched 2D LP solver: argument checks, context, dispatch.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rgb.h"
#include "rgb_internal.hpp"

namespace {

// Workspace of the solves issued on one stream (solves on one stream run in
// order, so they can share it).
struct WsSlot {
    void* stream = nullptr;
    void* mem = nullptr;
    int64_t cap = 0;
    rgb::Workspace ws{};
};

constexpr int kMaxStreams = 32;

}  // namespace

struct rgb_ctx {
    int device = 0;
    int num_cus = 0;
    int persist_blocks_per_cu = 1;
    rgb::PersistPlan plan{};
    std::vector<WsSlot> slots;
    std::string last_error;
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

// Makes ctx->device current for the lifetime of the guard.
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

constexpr int kDefaultLanes = 16;
constexpr int kDefaultChunk = 1;
constexpr int kDefaultDynFrac = 128;  // last 1/8 of the sub-batches go through the queue

// Lanes per LP by size class (class c holds 2^(c-1) < m <= 2^c).
void default_plan(rgb::PersistPlan& p) {
    for (int c = 0; c < rgb::kClasses; ++c) {
        int g = 64;
        if (c <= 4) g = 4;
        else if (c <= 6) g = 8;
        else if (c <= 8) g = 16;
        else if (c <= 9) g = 32;
        p.log2_lanes[c] = __builtin_ctz(g);
    }
    p.chunk = kDefaultChunk;
    p.dyn_frac_1024 = kDefaultDynFrac;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace for a solve of num_lps LPs on `stream`; grows with hipMalloc
// (never while the stream is being captured).
rgb_err_t get_workspace(rgb_ctx_t* ctx, void* stream, int64_t num_lps, rgb::Workspace& out) {
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
    if (slot->cap < num_lps || !slot->mem) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(reinterpret_cast<hipStream_t>(stream), &cs) == hipSuccess &&
            cs != hipStreamCaptureStatusNone)
            return fail(ctx, RGB_ERR_INVALID_ARG, "workspace must grow but the stream is being captured");
        int64_t cap = num_lps < 1024 ? 1024 : num_lps + num_lps / 4;
        static_assert(sizeof(rgb::QueueHeader) <= 1024, "queue header");
        static_assert(rgb::kQueues * rgb::kHeadStride * 4 <= 1024, "queue heads");
        size_t head_bytes = 2048;
        size_t blocks_off = head_bytes;
        size_t order_off = blocks_off + (size_t)rgb::kBinBlocks * rgb::kClasses * 4;
        size_t cls_off = align_up(order_off + (size_t)cap * 4, 256);
        size_t total = cls_off + align_up((size_t)cap, 256);
        if (slot->mem) {
            (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
            (void)hipFree(slot->mem);
            slot->mem = nullptr;
            slot->cap = 0;
        }
        void* mem = nullptr;
        if (hipMalloc(&mem, total) != hipSuccess) return fail(ctx, RGB_ERR_OOM, "workspace of %zu bytes", total);
        if (hipMemset(mem, 0, head_bytes) != hipSuccess) {
            (void)hipFree(mem);
            return fail(ctx, RGB_ERR_DEVICE, "workspace init failed");
        }
        char* base = static_cast<char*>(mem);
        slot->mem = mem;
        slot->cap = cap;
        slot->ws.q = reinterpret_cast<rgb::QueueHeader*>(base);
        slot->ws.heads = reinterpret_cast<int32_t*>(base + 1024);
        slot->ws.blocks = reinterpret_cast<int32_t*>(base + blocks_off);
        slot->ws.order = reinterpret_cast<int32_t*>(base + order_off);
        slot->ws.cls = reinterpret_cast<uint8_t*>(base + cls_off);
    }
    out = slot->ws;
    return RGB_OK;
}

}  // namespace

extern "C" {

const char* rgb_version(void) { return "rgb-mi355x 0.1 (gfx950)"; }

rgb_err_t rgb_ctx_create(int device, rgb_ctx_t** out) {
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
    ctx->persist_blocks_per_cu = rgb::persist_blocks_per_cu();
    default_plan(ctx->plan);
    *out = ctx;
    return RGB_OK;
}

rgb_err_t rgb_ctx_destroy(rgb_ctx_t* ctx) {
    if (!ctx) return RGB_OK;
    {
        DeviceGuard guard(ctx->device);
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

rgb_err_t rgb_solve_batch(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                          const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                          float* x_out, float* y_out, int32_t* status_out, const rgb_solve_opts_t* opts,
                          void* stream) {
    if (!ctx) return RGB_ERR_INVALID_ARG;
    ctx->last_error.clear();
    if (num_lps < 0 || num_constraints < 0)
        return fail(ctx, RGB_ERR_INVALID_ARG, "negative num_lps (%lld) or num_constraints (%lld)",
                    (long long)num_lps, (long long)num_constraints);
    if (num_lps == 0) return RGB_OK;
    if (!offsets || !cx || !cy || !x_out || !y_out || !status_out)
        return fail(ctx, RGB_ERR_INVALID_ARG, "null per-LP pointer");
    if (num_constraints > 0 && (!ax || !ay || !b)) return fail(ctx, RGB_ERR_INVALID_ARG, "null row pointer");
    if (num_lps > (int64_t)0x7fffffff) return fail(ctx, RGB_ERR_TOO_LARGE, "num_lps above 2^31-1");

    rgb_solve_opts_t o{};
    if (opts) o = *opts;
    int variant = o.variant;
    if (variant < RGB_VARIANT_AUTO || variant > RGB_VARIANT_BINNED)
        return fail(ctx, RGB_ERR_INVALID_ARG, "unknown variant %d", variant);

    rgb::Problem P{};
    P.offsets = offsets;
    P.ax = ax;
    P.ay = ay;
    P.b = b;
    P.cx = cx;
    P.cy = cy;
    P.x_out = x_out;
    P.y_out = y_out;
    P.status = status_out;
    P.n1d = o.n_1dlp_out;
    P.order = nullptr;
    P.num_lps = num_lps;
    P.num_constraints = num_constraints;

    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, RGB_ERR_DEVICE, "cannot select device %d", ctx->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (o.slots != 0) return fail(ctx, RGB_ERR_INVALID_ARG, "opts.slots is reserved and must be 0");
    hipEvent_t ev0 = reinterpret_cast<hipEvent_t>(o.ev_begin), ev1 = reinterpret_cast<hipEvent_t>(o.ev_end);
    if (variant == RGB_VARIANT_PLAIN) {
        if (ev0) (void)hipEventRecord(ev0, st);
        e = rgb::launch_plain(P, st);
        if (ev1) (void)hipEventRecord(ev1, st);
    } else if (variant == RGB_VARIANT_AUTO || variant == RGB_VARIANT_PERSISTENT || variant == RGB_VARIANT_BINNED) {
        if (o.chunk < 0 || o.grid < 0) return fail(ctx, RGB_ERR_INVALID_ARG, "negative chunk or grid");
        rgb::Workspace W;
        rgb_err_t rc = get_workspace(ctx, stream, num_lps, W);
        if (rc != RGB_OK) return rc;
        rgb::PersistPlan plan = ctx->plan;
        if (o.chunk) plan.chunk = o.chunk;
        if (o.queue_share < -1 || o.queue_share > 1024)
            return fail(ctx, RGB_ERR_INVALID_ARG, "queue_share %d outside [-1, 1024]", o.queue_share);
        if (o.queue_share) plan.dyn_frac_1024 = o.queue_share < 0 ? 0 : o.queue_share;
        if (o.lanes_per_lp) {
            if (!rgb::group_supported(o.lanes_per_lp))
                return fail(ctx, RGB_ERR_INVALID_ARG, "lanes_per_lp=%d is not one of 4, 8, 16, 32, 64", o.lanes_per_lp);
            for (int c = 0; c < rgb::kClasses; ++c) plan.log2_lanes[c] = __builtin_ctz(o.lanes_per_lp);
        }
        int grid = o.grid ? o.grid : ctx->num_cus * ctx->persist_blocks_per_cu;
        bool binned = variant == RGB_VARIANT_BINNED;
        e = rgb::launch_persistent(P, W, plan, grid, binned, st, reinterpret_cast<hipEvent_t>(o.ev_begin),
                                   reinterpret_cast<hipEvent_t>(o.ev_end));
    } else {
        int g = o.lanes_per_lp ? o.lanes_per_lp : kDefaultLanes;
        if (!rgb::group_supported(g))
            return fail(ctx, RGB_ERR_INVALID_ARG, "lanes_per_lp=%d is not one of 4, 8, 16, 32, 64", g);
        if (ev0) (void)hipEventRecord(ev0, st);
        e = rgb::launch_group(P, g, st);
        if (ev1) (void)hipEventRecord(ev1, st);
    }
    if (e != hipSuccess) return fail(ctx, RGB_ERR_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return RGB_OK;
}

}  // extern "C"
