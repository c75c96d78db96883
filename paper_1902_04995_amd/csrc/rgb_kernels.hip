// Solver kernels for batched 2D LPs on gfx950 (wave64).
//
// plain  - one LP per lane: the scan reads its rows one by one and the whole
//          1D LP runs serially in the lane.  This is the naive form of Sec. 3
//          (NaiveRGB): lanes of a wave violate at different rows, so the wave
//          runs every lane's 1D LP while most lanes idle.
// group  - G lanes (G = 4..64) per LP.  The scan tests the G rows after the
//          last violation at once and a ballot gives the first violated one;
//          its 1D LP (Eq. (3)-(4)) is split into work units over the G lanes
//          (Sec. 3), and u_left / u_right are combined with DPP min/max
//          instead of the paper's shared-memory atomics.  Rows are read with
//          coalesced loads and re-read from cache by later 1D LPs.
//
// Min/max are exact and order-free, and the row attaining a bound is found
// afterwards by recomputing the same bits (smallest index wins), so every
// kernel returns bit-identical results.
#include <hip/hip_runtime.h>

#include "rgb_device.hpp"
#include "rgb_internal.hpp"

namespace rgb {

// ---------------------------------------------------------------------------
// plain: one LP per lane
// ---------------------------------------------------------------------------
__device__ __forceinline__ int serial_find(const float* rax, const float* ray, const float* rb, int v, const Line& L,
                                           float target, bool up) {
    for (int h = 0; h < v; ++h) {
        float D;
        float s = wu_sigma(rax[h], ray[h], rb[h], L, D);
        if ((up ? D > 0.0f : D < 0.0f) && s == target) return h;
    }
    return kNoIdx;
}

__global__ __launch_bounds__(256) void k_plain(Problem P) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.num_lps) return;
    int64_t lp = P.order ? (int64_t)P.order[q] : q;
    int64_t start;
    int m;
    LpState st;
    float cx = P.cx[lp], cy = P.cy[lp];
    init_state(st, cx, cy);
    int n1d = 0;
    if (!lp_range(P, lp, start, m) || !__builtin_isfinite(cx) || !__builtin_isfinite(cy)) {
        set_dead(st, kInvalid);
        finish_lp(P, lp, start, st, 0, 0);
        return;
    }
    const float* rax = P.ax + start;
    const float* ray = P.ay + start;
    const float* rb = P.b + start;
    bool bad = false;
    int i = 0;
    for (; i < m && st.kind != kDead; ++i) {
        float ax = rax[i], ay = ray[i], b = rb[i];
        if (!finite3(ax, ay, b)) {
            bad = true;
            break;
        }
        if (!row_violates(ax, ay, b, st)) continue;
        ++n1d;
        if (ax == 0.0f && ay == 0.0f) {  // 0 <= b with b < 0
            set_dead(st, kInfeasible);
            break;
        }
        Line L;
        make_line(L, ax, ay, b);
        float hi = __builtin_huge_valf(), lo = -__builtin_huge_valf();
        bool par = false;
        for (int h = 0; h < i; ++h) work_unit(rax[h], ray[h], rb[h], L, hi, lo, par);
        if (par) {
            set_dead(st, kInfeasible);
            break;
        }
        if (!__builtin_isinf(hi) && !__builtin_isinf(lo)) {
            bool inf = lo > hi;
            if (near_tie(L, hi, lo)) {
                int il = serial_find(rax, ray, rb, i, L, lo, false);
                int ih = serial_find(rax, ray, rb, i, L, hi, true);
                if (il != kNoIdx && ih != kNoIdx)
                    inf = exact_lo_gt_hi(L, rax[il], ray[il], rb[il], rax[ih], ray[ih], rb[ih]);
            }
            if (inf) {
                set_dead(st, kInfeasible);
                break;
            }
        }
        move_on_line(st, i, L, hi, lo, prefers_up(L, cx, cy));
    }
    for (++i; i < m && !bad; ++i) bad = !finite3(rax[i], ray[i], rb[i]);
    if (bad) set_dead(st, kInvalid);
    int h = -1;
    if (st.kind == kPoint) {
        Line L;
        make_line(L, rax[st.l], ray[st.l], rb[st.l]);
        h = serial_find(rax, ray, rb, st.l, L, st.sig, st.up);
        if (h == kNoIdx) h = st.l;  // cannot happen (the bound came from these bits); x is NaN then
    }
    finish_lp(P, lp, start, st, h, n1d);
}

// ---------------------------------------------------------------------------
// group: G lanes per LP
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}

// Butterfly over aligned groups of G lanes: quad_perm xor 1 and xor 2, row
// half-mirror (8), row mirror (16), swizzle swap 16 (32), then the other half
// of the wave (64).
#define RGB_GROUP_REDUCE(NAME, T, OP, DPP)                                         \
    template <int G>                                                               \
    __device__ __forceinline__ T NAME(T v) {                                       \
        if constexpr (G >= 2) v = OP(v, DPP<0xB1>(v));                             \
        if constexpr (G >= 4) v = OP(v, DPP<0x4E>(v));                             \
        if constexpr (G >= 8) v = OP(v, DPP<0x141>(v));                            \
        if constexpr (G >= 16) v = OP(v, DPP<0x140>(v));                           \
        if constexpr (G >= 32) {                                                   \
            int s = __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F); \
            v = OP(v, __builtin_bit_cast(T, s));                                   \
        }                                                                          \
        if constexpr (G >= 64) v = OP(v, __shfl_xor(v, 32));                       \
        return v;                                                                  \
    }

__device__ __forceinline__ float fmin_(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float fmax_(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ int imin_(int a, int b) { return a < b ? a : b; }
RGB_GROUP_REDUCE(group_min, float, fmin_, dpp_f)
RGB_GROUP_REDUCE(group_max, float, fmax_, dpp_f)
RGB_GROUP_REDUCE(group_min_i, int, imin_, dpp_i)
#undef RGB_GROUP_REDUCE

template <int G>
__device__ __forceinline__ uint64_t group_mask(int gbase) {
    if constexpr (G == 64) return ~0ull;
    else return ((1ull << G) - 1ull) << gbase;
}

// Smallest row h < v of the LP whose bound on line L equals `target` on the
// given side; all G lanes of the group must be active.
template <int G>
__device__ __forceinline__ int group_find(const float* rax, const float* ray, const float* rb, int v, const Line& L,
                                          float target, bool up, int gl) {
    int best = kNoIdx;
    for (int h = gl; h < v; h += G) {
        float D;
        float s = wu_sigma(rax[h], ray[h], rb[h], L, D);
        bool hit = (up ? D > 0.0f : D < 0.0f) && s == target;
        best = (hit && h < best) ? h : best;
    }
    return group_min_i<G>(best);
}

template <int G>
__device__ __forceinline__ void solve_group(const Problem& P, int64_t lp) {
    const int lane = __lane_id();
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const uint64_t gmask = group_mask<G>(gbase);

    int64_t start = 0;
    int m = 0;
    float cx = 0.0f, cy = 0.0f;
    bool ok = false;
    if (lp >= 0) {
        cx = P.cx[lp];
        cy = P.cy[lp];
        ok = lp_range(P, lp, start, m) && __builtin_isfinite(cx) && __builtin_isfinite(cy);
    }
    const float* rax = P.ax + start;
    const float* ray = P.ay + start;
    const float* rb = P.b + start;

    LpState st;
    init_state(st, cx, cy);
    if (lp >= 0 && !ok) set_dead(st, kInvalid);
    bool done = lp < 0 || !ok || m == 0;
    bool bad = false;
    int cur = 0;
    int n1d = 0;

    while (__ballot(!done) != 0) {
        // scan window: rows cur .. cur+G-1
        int idx = cur + gl;
        bool in = !done && idx < m;
        float tx = 0.0f, ty = 0.0f, tb = 0.0f;
        if (in) {
            tx = rax[idx];
            ty = ray[idx];
            tb = rb[idx];
        }
        bool fin = finite3(tx, ty, tb);
        bad |= in && !fin;
        bool all_point = __ballot(in && st.kind != kPoint) == 0;
        bool viol;
        if (all_point) viol = in && point_violated(tx, ty, tb, st.px, st.py);
        else viol = in && fin && row_violates(tx, ty, tb, st);
        uint64_t bal = __ballot(viol) & gmask;
        if (bal == 0) {
            if (!done) {
                cur += G;
                if (cur >= m) done = true;
            }
        } else {
            int src = __builtin_ctzll(bal);
            int v = cur + (src - gbase);
            float lx = __shfl(tx, src);
            float ly = __shfl(ty, src);
            float lb = __shfl(tb, src);
            ++n1d;
            if (lx == 0.0f && ly == 0.0f) {  // 0 <= b with b < 0
                set_dead(st, kInfeasible);
            } else {
                Line L;
                make_line(L, lx, ly, lb);
                float hi = __builtin_huge_valf(), lo = -__builtin_huge_valf();
                bool par = false;
                for (int h = gl; h < v; h += G) work_unit(rax[h], ray[h], rb[h], L, hi, lo, par);
                hi = group_min<G>(hi);
                lo = group_max<G>(lo);
                par = (__ballot(par) & gmask) != 0;
                if (par) {
                    set_dead(st, kInfeasible);
                } else {
                    bool inf = false;
                    if (!__builtin_isinf(hi) && !__builtin_isinf(lo)) {
                        inf = lo > hi;
                        if (near_tie(L, hi, lo)) {
                            int il = group_find<G>(rax, ray, rb, v, L, lo, false, gl);
                            int ih = group_find<G>(rax, ray, rb, v, L, hi, true, gl);
                            if (il != kNoIdx && ih != kNoIdx)
                                inf = exact_lo_gt_hi(L, rax[il], ray[il], rb[il], rax[ih], ray[ih], rb[ih]);
                        }
                    }
                    if (inf) set_dead(st, kInfeasible);
                    else move_on_line(st, v, L, hi, lo, prefers_up(L, cx, cy));
                }
            }
            cur = v + 1;
            if (cur >= m || st.kind == kDead) done = true;
        }
    }
    // an LP that died early still gets its remaining rows checked for non-finite values
    if (lp >= 0 && st.kind == kDead && st.dead_status == kInfeasible)
        for (int idx = cur + gl; idx < m; idx += G) bad |= !finite3(rax[idx], ray[idx], rb[idx]);
    if ((__ballot(bad) & gmask) != 0) set_dead(st, kInvalid);

    int h = -1;
    if (__ballot(st.kind == kPoint) != 0) {
        if (st.kind == kPoint) {
            Line L;
            make_line(L, rax[st.l], ray[st.l], rb[st.l]);
            h = group_find<G>(rax, ray, rb, st.l, L, st.sig, st.up, gl);
            if (h == kNoIdx) h = st.l;  // cannot happen (the bound came from these bits); x is NaN then
        }
    }
    if (lp >= 0 && gl == 0) finish_lp(P, lp, start, st, h, n1d);
}

template <int G>
__global__ __launch_bounds__(256) void k_group(Problem P) {
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t q = (int64_t)blockIdx.x * LPS_PER_BLOCK + threadIdx.x / G;
    int64_t lp = -1;
    if (q < P.num_lps) lp = P.order ? (int64_t)P.order[q] : q;
    solve_group<G>(P, lp);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_plain(const Problem& P, hipStream_t stream) {
    if (P.num_lps == 0) return hipSuccess;
    int64_t blocks = (P.num_lps + 255) / 256;
    hipLaunchKernelGGL(k_plain, dim3((unsigned)blocks), dim3(256), 0, stream, P);
    return hipGetLastError();
}

template <int G>
static hipError_t launch_group_t(const Problem& P, hipStream_t stream) {
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t blocks = (P.num_lps + LPS_PER_BLOCK - 1) / LPS_PER_BLOCK;
    hipLaunchKernelGGL((k_group<G>), dim3((unsigned)blocks), dim3(256), 0, stream, P);
    return hipGetLastError();
}

bool group_supported(int g) {
    return g == 4 || g == 8 || g == 16 || g == 32 || g == 64;
}

hipError_t launch_group(const Problem& P, int g, hipStream_t stream) {
    if (P.num_lps == 0) return hipSuccess;
    switch (g) {
        case 4: return launch_group_t<4>(P, stream);
        case 8: return launch_group_t<8>(P, stream);
        case 16: return launch_group_t<16>(P, stream);
        case 32: return launch_group_t<32>(P, stream);
        case 64: return launch_group_t<64>(P, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rgb
