// Crowd time step kept on the device: the collision-avoidance use of batched
// 2D LPs that motivates the paper (each agent picks its velocity by an LP
// over half-planes from its neighbours).  One step, all on one stream:
//
//   grid      agents binned into square cells (count, scan, scatter);
//   build     one wave per agent: its k nearest other agents (exact, ordered
//             by FP32 squared distance, then index), one half-plane per
//             neighbour (unit normal towards it, offset half the distance
//             minus the radius), the speed disc |v| <= vmax as tangent
//             half-planes, all rows put in a random order (Seidel's method
//             wants one) given by SplitMix64 keys, written as the agent's LP;
//   solve     rgb_solve_batch with the preferred velocities as objectives;
//   integrate v = x* (0 for an infeasible LP), p += dt v, clamped to the room.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rgb.h"
#include "rgb_internal.hpp"

namespace {

constexpr int kMaxK = 64;      // neighbours per agent at most
constexpr int kMaxDisc = 63;   // speed-disc rows at most (k + disc <= 127)
constexpr int kCand = 256;     // candidate keys held per agent while searching
constexpr int kSlots = 128;    // row slots per agent
constexpr int kWaves = 4;      // agents per block
constexpr uint64_t kNone = ~0ull;

struct Grid {
    float x0, y0, x1, y1, h, inv_h;
    float fuzz;  // how far a rounded cell assignment can put a point outside its cell
    int W, H;
};

__device__ __forceinline__ int cell_of(float v, float v0, float inv_h, int n) {
    int c = (int)floorf((v - v0) * inv_h);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_grid_count(const float* px, const float* py, int64_t n, Grid g, int32_t* cell, int32_t* count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of(py[i], g.y0, g.inv_h, g.H) * g.W + cell_of(px[i], g.x0, g.inv_h, g.W);
    cell[i] = c;
    atomicAdd(&count[c], 1);
}

// Exclusive scan of count[0 .. C) into start[0 .. C] and cursor[0 .. C) in
// three passes over tiles of 1024 cells: tile sums, their scan (one block),
// then each tile's scan plus its offset.
constexpr int kTile = 1024;

__device__ __forceinline__ int32_t block_incl_scan(int32_t v, int32_t* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kTile; d <<= 1) {
        int32_t u = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    return sh[t];
}

__global__ __launch_bounds__(kTile) void k_scan_tiles(const int32_t* count, int64_t C, int32_t* tile_sum) {
    __shared__ int32_t sh[kTile];
    const int64_t c = (int64_t)blockIdx.x * kTile + threadIdx.x;
    const int32_t incl = block_incl_scan(c < C ? count[c] : 0, sh);
    if (threadIdx.x == kTile - 1) tile_sum[blockIdx.x] = incl;
}

// One block: exclusive scan of the tile sums in place, each thread over a run.
__global__ __launch_bounds__(kTile) void k_scan_tile_sums(int32_t* tile_sum, int64_t T, int32_t* start, int64_t C) {
    __shared__ int32_t sh[kTile];
    const int t = threadIdx.x;
    const int64_t per = (T + kTile - 1) / kTile;
    const int64_t lo = t * per, hi = lo + per < T ? lo + per : T;
    int32_t sum = 0;
    for (int64_t q = lo; q < hi; ++q) sum += tile_sum[q];
    int32_t run = block_incl_scan(sum, sh) - sum;
    for (int64_t q = lo; q < hi; ++q) {
        const int32_t v = tile_sum[q];
        tile_sum[q] = run;
        run += v;
    }
    if (t == kTile - 1) start[C] = run;
}

__global__ __launch_bounds__(kTile) void k_scan_apply(const int32_t* count, int64_t C, const int32_t* tile_sum,
                                                      int32_t* start, int32_t* cursor) {
    __shared__ int32_t sh[kTile];
    const int64_t c = (int64_t)blockIdx.x * kTile + threadIdx.x;
    const int32_t v = c < C ? count[c] : 0;
    const int32_t excl = block_incl_scan(v, sh) - v + tile_sum[blockIdx.x];
    if (c < C) {
        start[c] = excl;
        cursor[c] = excl;
    }
}

// Agents in cell order, with their positions next to them (one load each
// when a neighbour search walks a cell).
__global__ void k_grid_scatter(const int32_t* cell, const float* px, const float* py, int64_t n, int32_t* cursor,
                               int32_t* sorted, float* spx, float* spy) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int pos = atomicAdd(&cursor[cell[i]], 1);
    sorted[pos] = (int32_t)i;
    spx[pos] = px[i];
    spy[pos] = py[i];
}

// SplitMix64 (Steele, Lea and Flood 2014; constants as published by Vigna):
// the n-th output (n >= 1) of the generator seeded with s is mix(s + n G).
__device__ __forceinline__ uint64_t splitmix_nth(uint64_t seed, uint64_t n) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * n;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Keep the `keep` smallest of the first n keys (distinct), sorted, at the
// front: every lane holds H of them (H = 2 up to 128 keys, 4 up to 256) and
// counts how many keys are smaller (broadcast LDS reads, no chain of sort
// stages), then writes each kept key to its rank.
template <int H>
__device__ __forceinline__ void keep_by_rank(uint64_t* s, int n, int keep) {
    const int lane = __lane_id();
    uint64_t k[H];
    int r[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        k[h] = lane + 64 * h < n ? s[lane + 64 * h] : kNone;
        r[h] = 0;
    }
    for (int t = 0; t < n; ++t) {
        const uint64_t v = s[t];
#pragma unroll
        for (int h = 0; h < H; ++h) r[h] += v < k[h];
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
    for (int h = 0; h < H; ++h)
        if (lane + 64 * h < n && r[h] < keep) s[r[h]] = k[h];
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ int keep_best(uint64_t* s, int n, int keep) {
    if (n <= 64) keep_by_rank<1>(s, n, keep);
    else if (n <= 128) keep_by_rank<2>(s, n, keep);
    else keep_by_rank<4>(s, n, keep);
    return n < keep ? n : keep;
}

__global__ __launch_bounds__(64 * kWaves) void k_crowd_build(const float* px, const float* py, const int32_t* kk,
                                                             const int64_t* offsets, int64_t n, Grid g,
                                                             const int32_t* start, const int32_t* sorted,
                                                             const float* spx, const float* spy,
                                                             const float* disc, int n_disc, float radius,
                                                             uint64_t seed, int64_t step_host,
                                                             const int64_t* step_dev, float* ax, float* ay,
                                                             float* bb) {
    __shared__ uint64_t cand_all[kWaves][kCand];
    __shared__ uint64_t key_all[kWaves][kSlots];
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    const int64_t i = (int64_t)blockIdx.x * kWaves + w;
    if (i >= n) return;  // the whole wave
    uint64_t* cand = cand_all[w];
    const float pxi = px[i], pyi = py[i];
    const int ki = kk[i];
    const int cx = cell_of(pxi, g.x0, g.inv_h, g.W), cy = cell_of(pyi, g.y0, g.inv_h, g.H);
    const int rmax = max(max(max(cx, g.W - 1 - cx), max(cy, g.H - 1 - cy)), 2);

    // k nearest.  Cells are visited in batches, one cell per lane: first the
    // (2 R0 + 1)^2 block around the agent's cell, then one ring of cells at
    // Chebyshev distance r at a time (at most 64 cells per pass).  The lanes
    // walk their cells' members in step, so a batch costs as many loads in a
    // row as its fullest cell has members.  Agents beyond ring r are at least
    // r h away, so the search ends once the k-th best squared distance is
    // clearly below (r h)^2.
    constexpr int R0 = 2;
    constexpr int kBlockCells = (2 * R0 + 1) * (2 * R0 + 1);
    int nc = 0;
    uint64_t worst = kNone;  // k-th best key so far (once k are known): no larger key can be kept
    bool ready = false;      // cand[0 .. nc) is sorted and nc <= ki
    for (int r = R0; ; ++r) {
        const int first = r == R0;
        const int ncells = first ? kBlockCells : 8 * r;
        for (int base = 0; base < ncells; base += 64) {
            const int q = base + lane;
            int dx = 0, dy = 0;
            if (first) {
                dx = q % (2 * R0 + 1) - R0;
                dy = q / (2 * R0 + 1) - R0;
            } else if (q < 2 * r + 1) {  // bottom row
                dx = q - r;
                dy = -r;
            } else if (q < 4 * r + 2) {  // top row
                dx = q - (2 * r + 1) - r;
                dy = r;
            } else if (q < 6 * r + 1) {  // left column without corners
                dx = -r;
                dy = q - (4 * r + 2) - r + 1;
            } else {  // right column without corners
                dx = r;
                dy = q - (6 * r + 1) - r + 1;
            }
            const int X = cx + dx, Y = cy + dy;
            int s = 0, cnt = 0;
            if (q < ncells && X >= 0 && X < g.W && Y >= 0 && Y < g.H) {
                const int c = Y * g.W + X;
                s = start[c];
                cnt = start[c + 1] - s;
            }
            for (int m = 0; __ballot(m < cnt) != 0; ++m) {
                bool v = m < cnt;
                uint64_t key = kNone;
                if (v) {
                    const int j = sorted[s + m];
                    const float ddx = spx[s + m] - pxi, ddy = spy[s + m] - pyi;
                    const float d2 = ddx * ddx + ddy * ddy;
                    key = ((uint64_t)__builtin_bit_cast(uint32_t, d2) << 32) | (uint32_t)j;
                    v = j != (int)i && key < worst;
                }
                const uint64_t bal = __ballot(v);
                const int cntv = __popcll(bal);
                if (cntv > 0) ready = false;
                if (nc + cntv > kCand) nc = keep_best(cand, nc, ki);
                const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
                if (v) cand[nc + rank] = key;
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                nc += cntv;
            }
        }
        if (r >= rmax) break;  // every cell visited
        if (nc >= ki) {
            if (!ready) {
                nc = keep_best(cand, nc, ki);
                ready = true;
            }
            worst = cand[ki - 1];
            const float dk2 = __builtin_bit_cast(float, (uint32_t)(worst >> 32));
            const float lim = (float)r * g.h - 2.0f * g.fuzz;  // unvisited agents are farther than this
            if (lim > 0.0f && dk2 < lim * lim * 0.999999f) break;
        }
    }
    if (!ready) nc = keep_best(cand, nc, ki);  // sorted; nc == ki (the batch has more than ki agents)

    // rows: neighbours, then the speed disc; keys put them in random order.
    // A lane builds rows t = lane and t = lane + 64 in registers.  The keys
    // are distinct (their low 7 bits are t), so row t goes to position
    // rank(t) = #{s < m : key_s < key_t} of the ascending order: every lane
    // counts it over the m keys, each read once from LDS as a broadcast (no
    // dependent chain of sort stages), and stores its rows there directly.
    const int64_t step = step_host >= 0 ? step_host : *step_dev;
    const int m = ki + n_disc;
    uint64_t* key = key_all[w];
    float rx[2] = {0.0f, 0.0f}, ry[2] = {0.0f, 0.0f}, rb[2] = {0.0f, 0.0f};
    uint64_t kt[2] = {kNone, kNone};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        if (t < nc) {
            const int j = (int)(uint32_t)cand[t];
            const float ddx = px[j] - pxi, ddy = py[j] - pyi;
            const float dist = sqrtf(ddx * ddx + ddy * ddy);
            const bool zero = dist == 0.0f;
            rx[h] = zero ? 1.0f : ddx / dist;
            ry[h] = zero ? 0.0f : ddy / dist;
            rb[h] = 0.5f * (dist - radius);
        } else if (t >= ki && t < m) {
            rx[h] = disc[2 * (t - ki)];
            ry[h] = disc[2 * (t - ki) + 1];
            rb[h] = disc[2 * n_disc];
        }
        if (t < m) {
            const uint64_t ctr = ((uint64_t)step << 40) + ((uint64_t)i << 8) + (uint64_t)t;
            kt[h] = (splitmix_nth(seed, ctr + 1) & ~uint64_t(127)) | (uint64_t)t;
        }
        key[t] = kt[h];
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    int rank0 = 0, rank1 = 0;
    if (m <= 64) {  // one key per lane (most agents): half the compares
        for (int s = 0; s < m; ++s) rank0 += key[s] < kt[0];
    } else {
        for (int s = 0; s < m; ++s) {
            const uint64_t ks = key[s];
            rank0 += ks < kt[0];
            rank1 += ks < kt[1];
        }
    }
    const int64_t o = offsets[i];
    if (lane < m) {
        ax[o + rank0] = rx[0];
        ay[o + rank0] = ry[0];
        bb[o + rank0] = rb[0];
    }
    if (lane + 64 < m) {
        ax[o + rank1] = rx[1];
        ay[o + rank1] = ry[1];
        bb[o + rank1] = rb[1];
    }
}

__global__ void k_crowd_integrate(float* px, float* py, float* vx, float* vy, const int32_t* status, int64_t n,
                                  float dt, Grid g, int64_t* advance) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && advance) *advance += 1;  // the device step counter (read by this step's build)
    if (i >= n) return;
    float ux = vx[i], uy = vy[i];
    if (status[i] != 0) ux = uy = 0.0f;  // no feasible velocity: stand still
    vx[i] = ux;
    vy[i] = uy;
    const float sx = dt * ux, sy = dt * uy;
    float x = px[i] + sx, y = py[i] + sy;
    x = x < g.x0 ? g.x0 : (x > g.x1 ? g.x1 : x);
    y = y < g.y0 ? g.y0 : (y > g.y1 ? g.y1 : y);
    px[i] = x;
    py[i] = y;
}

}  // namespace

struct rgb_crowd {
    rgb_ctx_t* ctx = nullptr;
    int device = 0;
    int64_t n = 0, rows = 0, cells = 0;
    Grid g{};
    rgb_crowd_opts_t o{};
    char* mem = nullptr;
    int32_t* k = nullptr;
    int64_t* offsets = nullptr;
    float *ax = nullptr, *ay = nullptr, *b = nullptr, *disc = nullptr;
    int32_t *cell = nullptr, *count = nullptr, *start = nullptr, *cursor = nullptr, *sorted = nullptr;
    int32_t* tile_sum = nullptr;
    float *spx = nullptr, *spy = nullptr;
    int64_t* counter = nullptr;  // device step counter (step = -1)
};

extern "C" {

rgb_err_t rgb_crowd_create(rgb_ctx_t* ctx, int64_t n_agents, const int32_t* k, const float bounds[4],
                           const rgb_crowd_opts_t* opts, rgb_crowd_t** out) {
    if (!ctx || !k || !bounds || !out || n_agents < 2 || n_agents > (int64_t(1) << 30)) return RGB_ERR_INVALID_ARG;
    *out = nullptr;
    rgb_crowd_opts_t o{};
    if (opts) o = *opts;
    if (o.radius == 0.0f) o.radius = 0.3f;
    if (o.vmax == 0.0f) o.vmax = 1.0f;
    if (o.dt == 0.0f) o.dt = 0.1f;
    if (o.cell == 0.0f) o.cell = 2.0f;
    if (o.n_disc == 0) o.n_disc = 16;
    if (!(o.radius >= 0.0f) || !(o.vmax > 0.0f) || !(o.dt > 0.0f) || !(o.cell > 0.0f) || o.n_disc < 3 ||
        o.n_disc > kMaxDisc || !std::isfinite(o.radius) || !std::isfinite(o.vmax) || !std::isfinite(o.dt) ||
        !std::isfinite(o.cell))
        return RGB_ERR_INVALID_ARG;
    const float x0 = bounds[0], y0 = bounds[1], x1 = bounds[2], y1 = bounds[3];
    if (!std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(x1) || !std::isfinite(y1) || !(x1 > x0) ||
        !(y1 > y0))
        return RGB_ERR_INVALID_ARG;
    const double W = std::ceil((x1 - x0) / (double)o.cell), H = std::ceil((y1 - y0) / (double)o.cell);
    if (W * H > double(int64_t(1) << 26)) return RGB_ERR_INVALID_ARG;
    std::vector<int64_t> offs((size_t)n_agents + 1);
    offs[0] = 0;
    for (int64_t a = 0; a < n_agents; ++a) {
        if (k[a] < 1 || k[a] > kMaxK || k[a] > n_agents - 1) return RGB_ERR_INVALID_ARG;
        offs[a + 1] = offs[a] + k[a] + o.n_disc;
    }
    auto* c = new (std::nothrow) rgb_crowd();
    if (!c) return RGB_ERR_OOM;
    c->ctx = ctx;
    c->device = rgb::ctx_device(ctx);
    c->n = n_agents;
    c->rows = offs[(size_t)n_agents];
    c->o = o;
    c->g.x0 = x0;
    c->g.y0 = y0;
    c->g.x1 = x1;
    c->g.y1 = y1;
    c->g.h = o.cell;
    c->g.inv_h = 1.0f / o.cell;
    c->g.fuzz = (float)(4.0 * std::ldexp(1.0, -23) *
                        (std::max(std::max(std::fabs(x0), std::fabs(x1)), std::max(std::fabs(y0), std::fabs(y1))) +
                         o.cell));
    c->g.W = (int)std::max(1.0, W);
    c->g.H = (int)std::max(1.0, H);
    c->cells = (int64_t)c->g.W * c->g.H;
    // one allocation: k, offsets, rows, disc constants, grid arrays
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t n_ = (size_t)n_agents, R = (size_t)c->rows, C = (size_t)c->cells;
    const size_t sz_k = al(4 * n_), sz_off = al(8 * (n_ + 1)), sz_row = al(4 * R), sz_disc = al(4 * (2 * kMaxDisc + 1)),
                 sz_cell = al(4 * n_), sz_cnt = al(4 * (C + 1)), sz_sorted = al(4 * n_), sz_ctr = al(8),
                 sz_tiles = al(4 * ((C + kTile - 1) / kTile));
    const size_t total = sz_k + sz_off + 3 * sz_row + sz_disc + sz_cell + 3 * sz_cnt + 3 * sz_sorted + sz_ctr + sz_tiles;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) {
        delete c;
        return RGB_ERR_DEVICE;
    }
    if (c->device != prev && hipSetDevice(c->device) != hipSuccess) {
        delete c;
        return RGB_ERR_DEVICE;
    }
    rgb_err_t rc = RGB_OK;
    if (hipMalloc((void**)&c->mem, total) != hipSuccess) {
        c->mem = nullptr;
        rc = RGB_ERR_OOM;
    } else {
        char* p = c->mem;
        c->k = reinterpret_cast<int32_t*>(p); p += sz_k;
        c->offsets = reinterpret_cast<int64_t*>(p); p += sz_off;
        c->ax = reinterpret_cast<float*>(p); p += sz_row;
        c->ay = reinterpret_cast<float*>(p); p += sz_row;
        c->b = reinterpret_cast<float*>(p); p += sz_row;
        c->disc = reinterpret_cast<float*>(p); p += sz_disc;
        c->cell = reinterpret_cast<int32_t*>(p); p += sz_cell;
        c->count = reinterpret_cast<int32_t*>(p); p += sz_cnt;
        c->start = reinterpret_cast<int32_t*>(p); p += sz_cnt;
        c->cursor = reinterpret_cast<int32_t*>(p); p += sz_cnt;
        c->sorted = reinterpret_cast<int32_t*>(p); p += sz_sorted;
        c->spx = reinterpret_cast<float*>(p); p += sz_sorted;
        c->spy = reinterpret_cast<float*>(p); p += sz_sorted;
        c->tile_sum = reinterpret_cast<int32_t*>(p); p += sz_tiles;
        c->counter = reinterpret_cast<int64_t*>(p);
        // the disc: unit normals at angles 2 pi q / n_disc, offset vmax
        std::vector<float> disc(2 * kMaxDisc + 1, 0.0f);
        for (int q = 0; q < o.n_disc; ++q) {
            const double t = 2.0 * M_PI * q / o.n_disc;
            disc[2 * q] = (float)std::cos(t);
            disc[2 * q + 1] = (float)std::sin(t);
        }
        disc[2 * o.n_disc] = o.vmax;
        if (hipMemcpy(c->k, k, 4 * n_, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->offsets, offs.data(), 8 * (n_ + 1), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->disc, disc.data(), 4 * disc.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(c->counter, 0, 8) != hipSuccess ||
            // these run on the null stream, which a non-blocking stream does not
            // wait for: finish them before any step can be enqueued
            hipDeviceSynchronize() != hipSuccess)
            rc = RGB_ERR_DEVICE;
    }
    if (c->device != prev) (void)hipSetDevice(prev);
    if (rc != RGB_OK) {
        rgb_crowd_destroy(c);
        return rc;
    }
    *out = c;
    return RGB_OK;
}

rgb_err_t rgb_crowd_step(rgb_crowd_t* c, float* px, float* py, const float* gx, const float* gy, float* vx, float* vy,
                         int32_t* status, int64_t step, const rgb_solve_opts_t* opts, void* stream) {
    if (!c || !px || !py || !gx || !gy || !vx || !vy || !status || step < -1 || step >= (int64_t(1) << 23))
        return RGB_ERR_INVALID_ARG;
    if (opts && (opts->n_1dlp_out || opts->ev_begin || opts->ev_end)) return RGB_ERR_INVALID_ARG;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return RGB_ERR_DEVICE;
    if (c->device != prev && hipSetDevice(c->device) != hipSuccess) return RGB_ERR_DEVICE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = c->n, C = c->cells;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((C + 1 + 255) / 256)), dim3(256), 0, st, c->count, C + 1, 0);
    hipLaunchKernelGGL(k_grid_count, dim3(nb), dim3(256), 0, st, px, py, n, c->g, c->cell, c->count);
    const int64_t T = (C + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)T), dim3(kTile), 0, st, c->count, C, c->tile_sum);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kTile), 0, st, c->tile_sum, T, c->start, C);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)T), dim3(kTile), 0, st, c->count, C, c->tile_sum, c->start,
                       c->cursor);
    hipLaunchKernelGGL(k_grid_scatter, dim3(nb), dim3(256), 0, st, c->cell, px, py, n, c->cursor, c->sorted, c->spx,
                       c->spy);
    hipLaunchKernelGGL(k_crowd_build, dim3((unsigned)((n + kWaves - 1) / kWaves)), dim3(64 * kWaves), 0, st, px, py,
                       c->k, c->offsets, n, c->g, c->start, c->sorted, c->spx, c->spy, c->disc, c->o.n_disc,
                       c->o.radius, c->o.seed,
                       step, c->counter, c->ax, c->ay, c->b);
    rgb_err_t rc = hipGetLastError() == hipSuccess ? RGB_OK : RGB_ERR_DEVICE;
    if (rc == RGB_OK)
        rc = rgb_solve_batch(c->ctx, n, c->rows, c->offsets, c->ax, c->ay, c->b, gx, gy, vx, vy, status, opts,
                             stream);
    if (rc == RGB_OK) {
        hipLaunchKernelGGL(k_crowd_integrate, dim3(nb), dim3(256), 0, st, px, py, vx, vy, status, n, c->o.dt, c->g,
                           step < 0 ? c->counter : nullptr);
        if (hipGetLastError() != hipSuccess) rc = RGB_ERR_DEVICE;
    }
    if (c->device != prev) (void)hipSetDevice(prev);
    return rc;
}

rgb_err_t rgb_crowd_num_rows(const rgb_crowd_t* c, int64_t* num_constraints) {
    if (!c || !num_constraints) return RGB_ERR_INVALID_ARG;
    *num_constraints = c->rows;
    return RGB_OK;
}

rgb_err_t rgb_crowd_rows(const rgb_crowd_t* c, int64_t* offsets, float* ax, float* ay, float* b, void* stream) {
    if (!c || !offsets || !ax || !ay || !b) return RGB_ERR_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t R = 4 * (size_t)c->rows;
    bool ok = hipMemcpyAsync(offsets, c->offsets, 8 * (size_t)(c->n + 1), hipMemcpyDeviceToDevice, st) == hipSuccess &&
              hipMemcpyAsync(ax, c->ax, R, hipMemcpyDeviceToDevice, st) == hipSuccess &&
              hipMemcpyAsync(ay, c->ay, R, hipMemcpyDeviceToDevice, st) == hipSuccess &&
              hipMemcpyAsync(b, c->b, R, hipMemcpyDeviceToDevice, st) == hipSuccess;
    return ok ? RGB_OK : RGB_ERR_DEVICE;
}

rgb_err_t rgb_crowd_destroy(rgb_crowd_t* c) {
    if (!c) return RGB_OK;
    if (c->mem) {
        int prev = 0;
        const bool ok = hipGetDevice(&prev) == hipSuccess;
        if (ok && prev != c->device) (void)hipSetDevice(c->device);
        (void)hipFree(c->mem);
        if (ok && prev != c->device) (void)hipSetDevice(prev);
    }
    delete c;
    return RGB_OK;
}

}  // extern "C"
