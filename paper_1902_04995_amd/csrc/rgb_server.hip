// Served mode: continuous batching of LP requests over the solver ABI.
//
// rgb_server_submit copies a request once, into pinned host rings (one per
// input array), and queues it.  One scheduler thread owns every HIP call: it
// retires finished micro-batches (event polling), then, for each idle stream,
// takes queued requests in arrival order into a micro-batch while they sit
// next to each other in the rings and the LP cap and the arena's largest free
// block allow, copies the rings' spans straight into one arena block, solves
// it with rgb_solve_batch and copies the results back.
//
// Both copies are kernels on the slot's stream that read and write the
// pinned buffers directly, not DMA-engine copies: the copies, the solve and
// the completion event sit in one in-order queue.  The pinned buffers are
// fine-grained (coherent) host memory, so the GPU reads a reused ring span as
// the host last wrote it and its result stores are visible to the host when
// the kernel has finished.  The slots' streams are non-blocking, so nothing
// the server's solves depend on may be issued to the null stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rgb.h"
#include "arena.hpp"
#include "ring.hpp"
#include "rgb_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { kQueued = 0, kAdmitted = 1, kDone = 2, kFailed = 3 };

bool copy_words(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes % 4 != 0) return false;  // every region of a Layout is a whole number of 16-byte lines
    return rgb::launch_copy(dst, src, bytes, st);
}

struct Request {
    uint64_t id = 0;
    int64_t B = 0, N = 0;
    int64_t row_pos = 0, lp_pos = 0;  // first positions in the row and LP rings
    uint64_t row_blk = 0, lp_blk = 0;  // ring block ids
    bool ready = false;                // inputs copied into the rings
    std::vector<float> x, y;
    std::vector<int32_t> st;
    Clock::time_point t_submit, t_done;
    int state = kQueued;
};

// Byte layout of a micro-batch of B LPs and N rows (arena block and pinned
// staging buffer alike): inputs first (one host-to-device copy), then outputs
// (one device-to-host copy).
struct Layout {
    size_t offsets, cx, cy, ax, ay, b, in_bytes, x, y, st, total;
    static size_t al(size_t v) { return (v + 15) & ~size_t(15); }
    Layout(int64_t B, int64_t N) {
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

// Pinned buffer of a stream: the micro-batch's offsets on the way in, its
// x, y and status on the way out (the output part of Layout).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* pinned = nullptr;      // offsets: 8 (cap + 1) bytes, then the outputs
    char* pinned_dev = nullptr;  // the same buffer as the device sees it
    size_t out_at = 0;           // where the outputs start in `pinned`
    bool busy = false;
    uint64_t arena_off = 0;
    int64_t B = 0, N = 0;
    std::vector<Request*> reqs;
};

}  // namespace

struct rgb_server {
    int device = 0;
    rgb_ctx_t* ctx = nullptr;
    rgb_server_opts_t opts{};
    char* arena_mem = nullptr;
    rgb::Arena arena;
    std::vector<Slot> slots;
    // pinned request rings: rows (ax, ay, b) and LPs (cx, cy, end offset of
    // each LP relative to its request)
    char* ring_mem = nullptr;
    char* ring_dev = nullptr;  // ring_mem as the device sees it
    float *r_ax = nullptr, *r_ay = nullptr, *r_b = nullptr, *r_cx = nullptr, *r_cy = nullptr;
    int64_t* r_end = nullptr;
    rgb::Ring rows, lps;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_id = 1;
    rgb_server_stats_t stats{};
    bool stop = false;
    std::thread thr;

    void run();
    bool retire(Slot& s);
    bool launch(Slot& s);
};

// Finished micro-batch on slot s: copy results out, stamp, free the block.
bool rgb_server::retire(Slot& s) {
    hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) return false;
    Layout L(s.B, s.N);
    const char* out = s.pinned + s.out_at - L.x;  // outputs at the same offsets as in the arena block
    std::lock_guard<std::mutex> lk(mu);
    auto now = Clock::now();
    int64_t k = 0;
    for (Request* r : s.reqs) {
        rows.release(r->row_blk);
        lps.release(r->lp_blk);
        if (q == hipSuccess) {
            std::memcpy(r->x.data(), out + L.x + 4 * k, 4 * (size_t)r->B);
            std::memcpy(r->y.data(), out + L.y + 4 * k, 4 * (size_t)r->B);
            std::memcpy(r->st.data(), out + L.st + 4 * k, 4 * (size_t)r->B);
            r->state = kDone;
            stats.lps_completed += (uint64_t)r->B;
        } else {
            r->state = kFailed;
        }
        r->t_done = now;
        k += r->B;
        stats.completed++;
        stats.in_flight--;
    }
    arena.release(s.arena_off);
    stats.arena_bytes_in_use = arena.in_use();
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
    return true;
}

bool rgb_server::launch(Slot& s) {
    int64_t B = 0, N = 0;
    uint64_t off = UINT64_MAX;
    {
        std::lock_guard<std::mutex> lk(mu);
        const int64_t cap = opts.max_batch_lps;
        const uint64_t room = arena.largest_free();
        while (!queue.empty()) {
            Request* r = queue.front();
            if (!r->ready) break;
            if (opts.one_request_per_batch && !s.reqs.empty()) break;
            if (!s.reqs.empty()) {  // a micro-batch is one span of each ring
                const Request* p = s.reqs.back();
                if (r->row_pos != p->row_pos + p->N || r->lp_pos != p->lp_pos + p->B) break;
            }
            if (B + r->B > cap) break;
            if (arena.rounded(Layout(B + r->B, N + r->N).total) > room) break;
            queue.pop_front();
            s.reqs.push_back(r);
            B += r->B;
            N += r->N;
        }
        if (s.reqs.empty()) return false;
        off = arena.alloc(Layout(B, N).total);
        if (off == UINT64_MAX) {  // cannot happen: the block was sized against the largest free one
            for (auto it = s.reqs.rbegin(); it != s.reqs.rend(); ++it) queue.push_front(*it);
            s.reqs.clear();
            return false;
        }
        for (Request* r : s.reqs) r->state = kAdmitted;
        stats.pending = (int32_t)queue.size();
        stats.in_flight += (int32_t)s.reqs.size();
        stats.micro_batches++;
        stats.arena_bytes_in_use = arena.in_use();
        stats.arena_bytes_peak = std::max(stats.arena_bytes_peak, (uint64_t)arena.in_use());
    }
    Layout L(B, N);
    bool ok = true;
    {
        // offsets of the micro-batch: each request's LP ends shifted by its first row
        int64_t* offs = reinterpret_cast<int64_t*>(s.pinned);
        offs[0] = 0;
        int64_t lp = 0, row = 0;
        for (Request* r : s.reqs) {
            const int64_t* e = r_end + r->lp_pos;
            for (int64_t k = 0; k < r->B; ++k) offs[lp + k + 1] = row + e[k];
            lp += r->B;
            row += r->N;
        }
        const Request* f = s.reqs.front();
        char* d = arena_mem + off;
        // host pointer -> the same bytes as the device sees them
        auto dev_of = [&](const void* host) -> const void* {
            const char* h = static_cast<const char*>(host);
            if (h >= s.pinned && h < s.pinned + s.out_at) return s.pinned_dev + (h - s.pinned);
            return ring_dev + (h - ring_mem);
        };
        auto h2d = [&](size_t at, const void* src, size_t bytes) {
            if (ok && bytes) ok = copy_words(d + at, dev_of(src), bytes, s.stream);
        };
        h2d(L.offsets, offs, 8 * (size_t)(B + 1));
        h2d(L.cx, r_cx + f->lp_pos, 4 * (size_t)B);
        h2d(L.cy, r_cy + f->lp_pos, 4 * (size_t)B);
        h2d(L.ax, r_ax + f->row_pos, 4 * (size_t)N);
        h2d(L.ay, r_ay + f->row_pos, 4 * (size_t)N);
        h2d(L.b, r_b + f->row_pos, 4 * (size_t)N);
        if (ok) {
            rgb_solve_opts_t so{};
            so.variant = opts.variant;
            ok = rgb_solve_batch(ctx, B, N, reinterpret_cast<const int64_t*>(d + L.offsets),
                                 reinterpret_cast<const float*>(d + L.ax), reinterpret_cast<const float*>(d + L.ay),
                                 reinterpret_cast<const float*>(d + L.b), reinterpret_cast<const float*>(d + L.cx),
                                 reinterpret_cast<const float*>(d + L.cy), reinterpret_cast<float*>(d + L.x),
                                 reinterpret_cast<float*>(d + L.y), reinterpret_cast<int32_t*>(d + L.st), &so,
                                 s.stream) == RGB_OK;
        }
        if (ok) ok = copy_words(s.pinned_dev + s.out_at, d + L.x, L.total - L.x, s.stream);
        if (ok) ok = hipEventRecord(s.done, s.stream) == hipSuccess;
    }
    s.arena_off = off;
    s.B = B;
    s.N = N;
    s.busy = true;
    if (!ok) {
        (void)hipStreamSynchronize(s.stream);
        std::lock_guard<std::mutex> lk(mu);
        for (Request* r : s.reqs) {
            rows.release(r->row_blk);
            lps.release(r->lp_blk);
            r->state = kFailed;
            r->t_done = Clock::now();
            stats.completed++;
            stats.in_flight--;
        }
        arena.release(off);
        s.reqs.clear();
        s.busy = false;
        cv_done.notify_all();
    }
    return true;
}

void rgb_server::run() {
    (void)hipSetDevice(device);
    while (true) {
        bool progressed = false;
        bool any_busy = false;
        for (auto& s : slots)
            if (s.busy) progressed |= retire(s);
        {
            std::lock_guard<std::mutex> lk(mu);
            if (stop) break;
        }
        for (auto& s : slots)
            if (!s.busy) progressed |= launch(s);
        for (auto& s : slots) any_busy |= s.busy;
        if (progressed) continue;
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
        if (any_busy) cv_work.wait_for(lk, std::chrono::microseconds(20));
        else cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] { return stop || !queue.empty(); });
    }
    // drain: wait for the admitted micro-batches, then retire them
    for (auto& s : slots)
        if (s.busy) {
            (void)hipStreamSynchronize(s.stream);
            retire(s);
        }
}

extern "C" {

rgb_err_t rgb_server_create(rgb_ctx_t* ctx, const rgb_server_opts_t* opts, rgb_server_t** out) {
    if (!ctx || !out) return RGB_ERR_INVALID_ARG;
    *out = nullptr;
    rgb_server_opts_t o{};
    if (opts) o = *opts;
    if (o.hbm_budget == 0) o.hbm_budget = (uint64_t)1 << 30;
    if (o.n_streams == 0) o.n_streams = 4;
    if (o.max_batch_lps == 0) o.max_batch_lps = 65536;
    if (o.max_pending == 0) o.max_pending = 65536;
    if (o.host_ring_mib == 0) o.host_ring_mib = 256;
    if (o.n_streams < 1 || o.n_streams > 16 || o.max_batch_lps < 1 || o.max_pending < 1 || o.host_ring_mib < 1 ||
        o.host_ring_mib > (1 << 20) ||
        o.variant < RGB_VARIANT_AUTO || o.variant > RGB_VARIANT_POOLED || o.hbm_budget < 4096)
        return RGB_ERR_INVALID_ARG;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return RGB_ERR_DEVICE;
    const int dev = rgb::ctx_device(ctx);
    if (dev != prev && hipSetDevice(dev) != hipSuccess) return RGB_ERR_DEVICE;
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};
    rgb_server_t* s = new (std::nothrow) rgb_server_t();
    if (!s) return RGB_ERR_OOM;
    s->opts = o;
    s->device = dev;
    // the server's own context on ctx's device, with ctx's tuning
    rgb_tuning_t t;
    if (rgb_ctx_get_tuning(ctx, &t) != RGB_OK || rgb_ctx_create(dev, nullptr, &s->ctx) != RGB_OK ||
        rgb_ctx_set_tuning(s->ctx, &t) != RGB_OK) {
        rgb_server_destroy(s);
        return RGB_ERR_DEVICE;
    }
    if (hipMalloc((void**)&s->arena_mem, o.hbm_budget) != hipSuccess) {
        rgb_server_destroy(s);
        return RGB_ERR_OOM;
    }
    s->arena = rgb::Arena(o.hbm_budget, 256);
    // request rings: three quarters of the pinned bytes for rows (12 B each),
    // a quarter for LPs (16 B each)
    const size_t ring_bytes = (size_t)o.host_ring_mib << 20;
    const int64_t n_rows = (int64_t)(ring_bytes / 4 * 3 / 12), n_lps = (int64_t)(ring_bytes / 4 / 16);
    if (hipHostMalloc((void**)&s->ring_mem, (size_t)n_rows * 12 + (size_t)n_lps * 16,
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        s->ring_mem = nullptr;
        rgb_server_destroy(s);
        return RGB_ERR_OOM;
    }
    if (hipHostGetDevicePointer((void**)&s->ring_dev, s->ring_mem, 0) != hipSuccess) {
        rgb_server_destroy(s);
        return RGB_ERR_DEVICE;
    }
    // Touch every page of the rings once now: the first host write to a page
    // of this memory is several times slower than later ones, and without
    // this the first pass of requests through the rings (a whole ring's worth
    // of submits) pays it inside the submit calls.
    std::memset(s->ring_mem, 0, (size_t)n_rows * 12 + (size_t)n_lps * 16);
    s->r_end = reinterpret_cast<int64_t*>(s->ring_mem);
    s->r_cx = reinterpret_cast<float*>(s->r_end + n_lps);
    s->r_cy = s->r_cx + n_lps;
    s->r_ax = s->r_cy + n_lps;
    s->r_ay = s->r_ax + n_rows;
    s->r_b = s->r_ay + n_rows;
    s->rows = rgb::Ring(n_rows);
    s->lps = rgb::Ring(n_lps);
    s->slots.resize((size_t)o.n_streams);
    const size_t cap = (size_t)o.max_batch_lps;
    for (auto& sl : s->slots) {
        sl.out_at = Layout::al(8 * (cap + 1));
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&sl.pinned, sl.out_at + 3 * Layout::al(4 * cap),
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            sl.pinned = nullptr;
            rgb_server_destroy(s);
            return RGB_ERR_DEVICE;
        }
        if (hipHostGetDevicePointer((void**)&sl.pinned_dev, sl.pinned, 0) != hipSuccess) {
            rgb_server_destroy(s);
            return RGB_ERR_DEVICE;
        }
        std::memset(sl.pinned, 0, sl.out_at + 3 * Layout::al(4 * cap));
        // the solver's workspace for this stream at its largest micro-batch
        // now, not by reallocation (which synchronises) while serving
        if (!rgb::reserve_workspace(s->ctx, sl.stream, cap)) {
            rgb_server_destroy(s);
            return RGB_ERR_OOM;
        }
    }
    s->thr = std::thread([s] { s->run(); });
    *out = s;
    return RGB_OK;
}

rgb_err_t rgb_server_submit(rgb_server_t* srv, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                            const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                            uint64_t* ticket) {
    if (!srv || !ticket || num_lps < 0 || num_constraints < 0 || !offsets) return RGB_ERR_INVALID_ARG;
    if (num_lps > 0 && (!cx || !cy)) return RGB_ERR_INVALID_ARG;
    if (num_constraints > 0 && (!ax || !ay || !b)) return RGB_ERR_INVALID_ARG;
    auto t0 = Clock::now();
    if (num_lps > srv->opts.max_batch_lps || num_constraints > srv->rows.capacity() ||
        num_lps > srv->lps.capacity() ||
        srv->arena.rounded(Layout(num_lps, num_constraints).total) > srv->arena.capacity()) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stats.rejected_too_large++;
        return RGB_ERR_TOO_LARGE;
    }
    // offsets must tile [0, num_constraints): a request reads only its own rows
    // even after it is packed into a micro-batch with others
    if (offsets[0] != 0 || offsets[num_lps] != num_constraints) return RGB_ERR_INVALID_ARG;
    for (int64_t k = 0; k < num_lps; ++k)
        if (offsets[k + 1] < offsets[k]) return RGB_ERR_INVALID_ARG;
    auto r = std::make_unique<Request>();
    r->B = num_lps;
    r->N = num_constraints;
    r->x.resize((size_t)num_lps);
    r->y.resize((size_t)num_lps);
    r->st.resize((size_t)num_lps);
    r->t_submit = t0;
    Request* q = r.get();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        bool room = (int64_t)srv->queue.size() < srv->opts.max_pending;
        if (room && !srv->lps.alloc(num_lps, q->lp_pos, q->lp_blk)) room = false;
        if (room && !srv->rows.alloc(num_constraints, q->row_pos, q->row_blk)) {
            srv->lps.release(q->lp_blk);
            room = false;
        }
        if (!room) {
            srv->stats.rejected_busy++;
            return RGB_ERR_BUSY;
        }
        q->id = srv->next_id++;
        *ticket = q->id;
        srv->queue.push_back(q);  // not ready yet: the scheduler stops in front of it
        srv->reqs[q->id] = std::move(r);
        srv->stats.submitted++;
        srv->stats.pending = (int32_t)srv->queue.size();
    }
    // the one copy of the request, outside the lock, into its ring blocks
    if (num_lps > 0) {
        int64_t* e = srv->r_end + q->lp_pos;
        for (int64_t k = 0; k < num_lps; ++k) e[k] = offsets[k + 1];
        std::memcpy(srv->r_cx + q->lp_pos, cx, 4 * (size_t)num_lps);
        std::memcpy(srv->r_cy + q->lp_pos, cy, 4 * (size_t)num_lps);
    }
    if (num_constraints > 0) {
        std::memcpy(srv->r_ax + q->row_pos, ax, 4 * (size_t)num_constraints);
        std::memcpy(srv->r_ay + q->row_pos, ay, 4 * (size_t)num_constraints);
        std::memcpy(srv->r_b + q->row_pos, b, 4 * (size_t)num_constraints);
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        q->ready = true;
    }
    srv->cv_work.notify_one();
    return RGB_OK;
}

rgb_err_t rgb_server_poll(rgb_server_t* srv, uint64_t ticket, int32_t wait_ms, float* x_out, float* y_out,
                          int32_t* status_out, double* latency_ms, int32_t* done) {
    if (!srv || !done) return RGB_ERR_INVALID_ARG;
    *done = 0;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return RGB_ERR_NOT_FOUND;
    Request* r = it->second.get();
    auto finished = [&] { return r->state == kDone || r->state == kFailed; };
    if (!finished() && wait_ms != 0) {
        if (wait_ms < 0) srv->cv_done.wait(lk, finished);
        else srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), finished);
    }
    if (!finished()) return RGB_OK;
    if (r->B > 0 && (!x_out || !y_out || !status_out)) return RGB_ERR_INVALID_ARG;
    rgb_err_t rc = RGB_OK;
    if (r->state == kDone) {
        std::memcpy(x_out, r->x.data(), 4 * (size_t)r->B);
        std::memcpy(y_out, r->y.data(), 4 * (size_t)r->B);
        std::memcpy(status_out, r->st.data(), 4 * (size_t)r->B);
    } else {
        rc = RGB_ERR_DEVICE;
    }
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    *done = 1;
    srv->reqs.erase(it);
    return rc;
}

rgb_err_t rgb_server_stats(rgb_server_t* srv, rgb_server_stats_t* out) {
    if (!srv || !out) return RGB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    return RGB_OK;
}

rgb_err_t rgb_server_destroy(rgb_server_t* srv) {
    if (!srv) return RGB_OK;
    if (srv->thr.joinable()) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv_work.notify_all();
        srv->thr.join();
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (Request* r : srv->queue) {
            r->state = kFailed;
            r->t_done = Clock::now();
        }
        srv->queue.clear();
    }
    srv->cv_done.notify_all();
    for (auto& sl : srv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    if (srv->ring_mem) (void)hipHostFree(srv->ring_mem);
    if (srv->arena_mem) (void)hipFree(srv->arena_mem);
    if (srv->ctx) rgb_ctx_destroy(srv->ctx);
    delete srv;
    return RGB_OK;
}

}  // extern "C"
