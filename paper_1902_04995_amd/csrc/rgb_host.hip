// Host-to-host solve: a batch in host memory is cut into chunks of whole LPs
// and pushed through three streams, so that chunk k+1's copies overlap chunk
// k's solve.  Per chunk and stream: inputs to the device (straight from the
// caller's buffers when they are pinned, else through a pinned staging
// buffer filled by several host threads), the chunk's offsets rebased to its
// first row, rgb_solve_batch, results back.  The state (streams, device and
// pinned buffers) lives in the context and grows on demand.
//
// Every copy is a kernel on the chunk's stream that reads or writes the host
// buffer through its device-visible address (launch_copy), never a DMA-engine
// copy: the host waits on an event recorded after the results' copy, and a
// completion marker that follows a kernel on the same in-order queue has
// covered every store of that kernel.  The served path moved to kernel
// copies after a completed event that followed DMA copies was observed
// before the results had reached host memory; this path shares the
// mechanism.  The staging buffers are fine-grained (coherent) pinned memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/rgb.h"
#include "rgb_internal.hpp"

namespace rgb {

namespace {

constexpr int kHostStreams = 3;

// Byte layout of one chunk of B LPs and N rows, in the device buffer and the
// staging buffer alike: inputs, then outputs.
struct ChunkLayout {
    size_t offsets, cx, cy, ax, ay, b, in_bytes, x, y, st, total;
    static size_t al(size_t v) { return (v + 255) & ~size_t(255); }
    ChunkLayout(int64_t B, int64_t N) {
        size_t p = 0;
        offsets = p; p = al(p + 8 * (size_t)(B + 1));
        cx = p; p = al(p + 4 * (size_t)B);
        cy = p; p = al(p + 4 * (size_t)B);
        ax = p; p = al(p + 4 * (size_t)N);
        ay = p; p = al(p + 4 * (size_t)N);
        b = p; p = al(p + 4 * (size_t)N);
        in_bytes = p;
        x = p; p = al(p + 4 * (size_t)B);
        y = p; p = al(p + 4 * (size_t)B);
        st = p; p = al(p + 4 * (size_t)B);
        total = p;
    }
};

struct HostSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* dev = nullptr;
    size_t dev_cap = 0;
    char* pin = nullptr;      // fine-grained pinned staging buffer
    char* pin_dev = nullptr;  // the same buffer as the device sees it
    size_t pin_cap = 0;
    // the chunk in flight on this slot (its results still to be copied out)
    bool busy = false;
    int64_t lp0 = 0, B = 0, N = 0;
};

__global__ __launch_bounds__(256) void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_copy4(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                               int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_copy1(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src,
                                               int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_rebase(int64_t* offs, int64_t n, int64_t base) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) offs[i] -= base;
}

// Is p pinned host memory?  Then *dev receives the address a kernel uses for
// it (nullptr stays nullptr).
bool pinned_dev(const void* p, const char** dev) {
    *dev = nullptr;
    if (!p) return true;  // nothing to copy
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable memory is reported as an error: clear it
        return false;
    }
    if (a.type != hipMemoryTypeHost || !a.devicePointer) return false;
    *dev = static_cast<const char*>(a.devicePointer);
    return true;
}

// memcpy split over a few host threads for large copies.
void par_copy(void* dst, const void* src, size_t bytes) {
    const size_t kPiece = size_t(4) << 20;
    unsigned nt = (unsigned)std::min<size_t>(8, bytes / kPiece);
    if (nt <= 1) {
        if (bytes) std::memcpy(dst, src, bytes);
        return;
    }
    std::vector<std::thread> th;
    const size_t per = (bytes + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        size_t lo = t * per, hi = std::min(bytes, lo + per);
        if (lo >= hi) break;
        th.emplace_back([=] { std::memcpy((char*)dst + lo, (const char*)src + lo, hi - lo); });
    }
    for (auto& t : th) t.join();
}

}  // namespace

bool launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return true;
    const uintptr_t a = reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src);
    int64_t n;
    int width;
    if ((a % 16) == 0 && bytes % 16 == 0) {
        n = (int64_t)(bytes / 16);
        width = 16;
    } else if ((a % 4) == 0 && bytes % 4 == 0) {
        n = (int64_t)(bytes / 4);
        width = 4;
    } else {
        n = (int64_t)bytes;
        width = 1;
    }
    // enough waves in flight for host memory's latency, at most 4096 blocks
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (width == 16)
        hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, stream, static_cast<uint4*>(dst),
                           static_cast<const uint4*>(src), n);
    else if (width == 4)
        hipLaunchKernelGGL(k_copy4, dim3(blocks), dim3(256), 0, stream, static_cast<uint32_t*>(dst),
                           static_cast<const uint32_t*>(src), n);
    else
        hipLaunchKernelGGL(k_copy1, dim3(blocks), dim3(256), 0, stream, static_cast<uint8_t*>(dst),
                           static_cast<const uint8_t*>(src), n);
    return hipGetLastError() == hipSuccess;
}

struct HostPath {
    HostSlot slot[kHostStreams];
};

void destroy_host_path(HostPath* h) {
    if (!h) return;
    for (auto& s : h->slot) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.dev) (void)hipFree(s.dev);
        if (s.pin) (void)hipHostFree(s.pin);
    }
    delete h;
}

}  // namespace rgb

using rgb::ChunkLayout;
using rgb::HostSlot;

extern "C" rgb_err_t rgb_solve_batch_host(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints,
                                          const int64_t* offsets, const float* ax, const float* ay, const float* b,
                                          const float* cx, const float* cy, float* x_out, float* y_out,
                                          int32_t* status_out, const rgb_solve_opts_t* opts, int64_t chunk_rows,
                                          double* ms_out) {
    if (!ctx) return RGB_ERR_INVALID_ARG;
    if (num_lps < 0 || num_constraints < 0 || !offsets || chunk_rows < 0) return RGB_ERR_INVALID_ARG;
    if (num_lps > 0 && (!cx || !cy || !x_out || !y_out || !status_out)) return RGB_ERR_INVALID_ARG;
    if (num_constraints > 0 && (!ax || !ay || !b)) return RGB_ERR_INVALID_ARG;
    // per-call device outputs and event hooks do not apply to a chunked solve
    if (opts && (opts->n_1dlp_out || opts->ev_begin || opts->ev_end)) return RGB_ERR_INVALID_ARG;
    // chunks are cut at LP boundaries, so the offsets must be in range and non-decreasing
    if (offsets[0] < 0 || offsets[num_lps] > num_constraints) return RGB_ERR_INVALID_ARG;
    for (int64_t k = 0; k < num_lps; ++k)
        if (offsets[k + 1] < offsets[k]) return RGB_ERR_INVALID_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    if (num_lps == 0) {
        if (ms_out) *ms_out = 0.0;
        return RGB_OK;
    }
    if (chunk_rows == 0) chunk_rows = int64_t(8) << 20;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return RGB_ERR_DEVICE;
    const int dev = rgb::ctx_device(ctx);
    if (dev != prev && hipSetDevice(dev) != hipSuccess) return RGB_ERR_DEVICE;
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};

    rgb::HostPath*& hp = rgb::ctx_host_path(ctx);
    if (!hp) {
        hp = new (std::nothrow) rgb::HostPath();
        if (!hp) return RGB_ERR_OOM;
        for (auto& s : hp->slot)
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
                return RGB_ERR_DEVICE;
    }
    // device-visible addresses of the caller's buffers where they are pinned
    const char *d_off, *d_ax, *d_ay, *d_b, *d_cx, *d_cy, *d_x, *d_y, *d_st;
    const bool pin_in = rgb::pinned_dev(offsets, &d_off) && rgb::pinned_dev(ax, &d_ax) && rgb::pinned_dev(ay, &d_ay) &&
                        rgb::pinned_dev(b, &d_b) && rgb::pinned_dev(cx, &d_cx) && rgb::pinned_dev(cy, &d_cy);
    const bool pin_out =
        rgb::pinned_dev(x_out, &d_x) && rgb::pinned_dev(y_out, &d_y) && rgb::pinned_dev(status_out, &d_st);

    rgb_err_t rc = RGB_OK;
    // results of a finished chunk, from the staging buffer to the caller
    auto drain = [&](HostSlot& s) {
        if (!s.busy) return;
        if (hipEventSynchronize(s.done) != hipSuccess) rc = RGB_ERR_DEVICE;
        if (!pin_out && rc == RGB_OK) {
            ChunkLayout L(s.B, s.N);
            std::memcpy(x_out + s.lp0, s.pin + L.x, 4 * (size_t)s.B);
            std::memcpy(y_out + s.lp0, s.pin + L.y, 4 * (size_t)s.B);
            std::memcpy(status_out + s.lp0, s.pin + L.st, 4 * (size_t)s.B);
        }
        s.busy = false;
    };
    int64_t lp0 = 0;
    int k = 0;
    while (lp0 < num_lps && rc == RGB_OK) {
        // the chunk: whole LPs up to chunk_rows rows (at least one LP)
        const int64_t row0 = offsets[lp0];
        int64_t lp1 = std::upper_bound(offsets + lp0 + 1, offsets + num_lps + 1, row0 + chunk_rows) - offsets - 1;
        if (lp1 <= lp0) lp1 = lp0 + 1;
        const int64_t B = lp1 - lp0, N = offsets[lp1] - row0;
        HostSlot& s = hp->slot[k % rgb::kHostStreams];
        drain(s);
        if (rc != RGB_OK) break;
        ChunkLayout L(B, N);
        if (s.dev_cap < L.total) {
            if (s.dev) (void)hipFree(s.dev);
            s.dev = nullptr;
            s.dev_cap = 0;
            if (hipMalloc((void**)&s.dev, L.total) != hipSuccess) {
                rc = RGB_ERR_OOM;
                break;
            }
            s.dev_cap = L.total;
        }
        const bool need_pin = !pin_in || !pin_out;
        if (need_pin && s.pin_cap < L.total) {
            if (s.pin) (void)hipHostFree(s.pin);
            s.pin = nullptr;
            s.pin_dev = nullptr;
            s.pin_cap = 0;
            if (hipHostMalloc((void**)&s.pin, L.total, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
                s.pin = nullptr;
                rc = RGB_ERR_OOM;
                break;
            }
            if (hipHostGetDevicePointer((void**)&s.pin_dev, s.pin, 0) != hipSuccess) {
                rc = RGB_ERR_DEVICE;
                break;
            }
            s.pin_cap = L.total;
        }
        // inputs: offsets (rebased on the device), objectives, rows, read by
        // copy kernels through the device-visible address of the caller's
        // pinned buffers or of the staging buffer
        const char* src_off = d_off + 8 * lp0;
        const char* src_cx = d_cx + 4 * lp0;
        const char* src_cy = d_cy + 4 * lp0;
        const char* src_ax = d_ax + 4 * row0;
        const char* src_ay = d_ay + 4 * row0;
        const char* src_b = d_b + 4 * row0;
        if (!pin_in) {
            rgb::par_copy(s.pin + L.offsets, offsets + lp0, 8 * (size_t)(B + 1));
            rgb::par_copy(s.pin + L.cx, cx + lp0, 4 * (size_t)B);
            rgb::par_copy(s.pin + L.cy, cy + lp0, 4 * (size_t)B);
            rgb::par_copy(s.pin + L.ax, ax + row0, 4 * (size_t)N);
            rgb::par_copy(s.pin + L.ay, ay + row0, 4 * (size_t)N);
            rgb::par_copy(s.pin + L.b, b + row0, 4 * (size_t)N);
            src_off = s.pin_dev + L.offsets;
            src_cx = s.pin_dev + L.cx;
            src_cy = s.pin_dev + L.cy;
            src_ax = s.pin_dev + L.ax;
            src_ay = s.pin_dev + L.ay;
            src_b = s.pin_dev + L.b;
        }
        bool ok = true;
        auto h2d = [&](size_t at, const char* src, size_t bytes) {
            if (ok && bytes) ok = rgb::launch_copy(s.dev + at, src, bytes, s.stream);
        };
        h2d(L.offsets, src_off, 8 * (size_t)(B + 1));
        h2d(L.cx, src_cx, 4 * (size_t)B);
        h2d(L.cy, src_cy, 4 * (size_t)B);
        h2d(L.ax, src_ax, 4 * (size_t)N);
        h2d(L.ay, src_ay, 4 * (size_t)N);
        h2d(L.b, src_b, 4 * (size_t)N);
        if (ok && row0 != 0) {
            hipLaunchKernelGGL(rgb::k_rebase, dim3((unsigned)((B + 256) / 256)), dim3(256), 0, s.stream,
                               reinterpret_cast<int64_t*>(s.dev + L.offsets), B + 1, row0);
            ok = hipGetLastError() == hipSuccess;
        }
        if (ok) {
            rgb_err_t e = rgb_solve_batch(ctx, B, N, reinterpret_cast<const int64_t*>(s.dev + L.offsets),
                                          reinterpret_cast<const float*>(s.dev + L.ax),
                                          reinterpret_cast<const float*>(s.dev + L.ay),
                                          reinterpret_cast<const float*>(s.dev + L.b),
                                          reinterpret_cast<const float*>(s.dev + L.cx),
                                          reinterpret_cast<const float*>(s.dev + L.cy),
                                          reinterpret_cast<float*>(s.dev + L.x), reinterpret_cast<float*>(s.dev + L.y),
                                          reinterpret_cast<int32_t*>(s.dev + L.st), opts, s.stream);
            if (e != RGB_OK) {
                rc = e;
                break;
            }
        }
        if (ok) {
            if (pin_out) {
                ok = rgb::launch_copy(const_cast<char*>(d_x) + 4 * lp0, s.dev + L.x, 4 * (size_t)B, s.stream) &&
                     rgb::launch_copy(const_cast<char*>(d_y) + 4 * lp0, s.dev + L.y, 4 * (size_t)B, s.stream) &&
                     rgb::launch_copy(const_cast<char*>(d_st) + 4 * lp0, s.dev + L.st, 4 * (size_t)B, s.stream);
            } else {
                ok = rgb::launch_copy(s.pin_dev + L.x, s.dev + L.x, L.total - L.x, s.stream);
            }
        }
        if (ok) ok = hipEventRecord(s.done, s.stream) == hipSuccess;
        if (!ok) {
            rc = RGB_ERR_DEVICE;
            break;
        }
        s.busy = true;
        s.lp0 = lp0;
        s.B = B;
        s.N = N;
        lp0 = lp1;
        ++k;
    }
    for (auto& s : hp->slot) {
        if (rc == RGB_OK) {
            drain(s);
        } else {  // nothing may still read or write the caller's buffers after the return
            (void)hipStreamSynchronize(s.stream);
            s.busy = false;
        }
    }
    if (ms_out) *ms_out = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}
