// C ABI of the batched 2D LP solver: argument checks, context, dispatch.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/rgb.h"
#include "rgb_internal.hpp"

struct rgb_ctx {
    int device;
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
    *out = ctx;
    return RGB_OK;
}

rgb_err_t rgb_ctx_destroy(rgb_ctx_t* ctx) {
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
    if (variant < RGB_VARIANT_AUTO || variant > RGB_VARIANT_PERSISTENT)
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
    if (variant == RGB_VARIANT_PLAIN) {
        e = rgb::launch_plain(P, st);
    } else {
        int g = o.lanes_per_lp ? o.lanes_per_lp : kDefaultLanes;
        if (!rgb::group_supported(g))
            return fail(ctx, RGB_ERR_INVALID_ARG, "lanes_per_lp=%d is not one of 4, 8, 16, 32, 64", g);
        e = rgb::launch_group(P, g, st);
    }
    if (e != hipSuccess) return fail(ctx, RGB_ERR_DEVICE, "launch failed: %s", hipGetErrorString(e));
    return RGB_OK;
}

}  // extern "C"
