// Solver kernels for batched 2D LPs on gfx950 (wave64).
//
// plain   - one LP per lane, rows read from memory as the scan reaches
//           them, the whole 1D LP serial in the lane.  This is the naive
//           form of Sec. 3 (NaiveRGB): lanes of a wave violate at different
//           steps, so the wave runs every lane's 1D LP with most lanes idle.
// group   - G lanes (G = 4..64) per LP.  The LP's rows are loaded once,
//           coalesced, into registers: row j lives in lane j % G, slot j / G.
//           The scan tests G rows at a time against the current state and a
//           ballot gives the first violated row; its 1D LP (Eq. (3)-(4)) is
//           split into work units over the G lanes (Sec. 3) and the bounds
//           are combined with cross-lane min/max instead of the paper's
//           shared-memory atomics.  Since a min/max with a smallest-index
//           tie-break is exact and order free, every variant returns bit-
//           identical results.  Rows beyond G*S are read from memory.
#include <hip/hip_runtime.h>

#include "rgb_device.hpp"
#include "rgb_internal.hpp"

namespace rgb {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// plain: one LP per lane
// ---------------------------------------------------------------------------
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
        st.kind = kDead;
        st.dead_status = kInvalid;
        finish_lp(P, lp, start, st, 0);
        return;
    }
    const float* rax = P.ax + start;
    const float* ray = P.ay + start;
    const float* rb = P.b + start;
    for (int i = 0; i < m; ++i) {
        if (!finite3(rax[i], ray[i], rb[i])) {
            st.kind = kDead;
            st.dead_status = kInvalid;
            break;
        }
    }
    for (int i = 0; i < m && st.kind != kDead; ++i) {
        float ax = rax[i], ay = ray[i], b = rb[i];
        if (!row_violates(ax, ay, b, st)) continue;
        ++n1d;
        if (ax == 0.0f && ay == 0.0f) {  // 0 <= b with b < 0
            st.kind = kDead;
            st.dead_status = kInfeasible;
            break;
        }
        Line L;
        make_line(L, ax, ay, b);
        Bounds B;
        init_bounds(B);
        for (int h = 0; h < i; ++h) work_unit(rax[h], ray[h], rb[h], h, L, B);
        apply_1dlp(st, i, L, B, cx, cy, rax, ray, rb);
    }
    finish_lp(P, lp, start, st, n1d);
}

// ---------------------------------------------------------------------------
// group: G lanes per LP, S register slots per lane
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ uint64_t group_mask(int gbase) {
    if constexpr (G == 64) return ~0ull;
    else return ((1ull << G) - 1ull) << gbase;
}

template <int G>
__device__ __forceinline__ void group_reduce(Bounds& B) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        float ohi = __shfl_xor(B.hi, off, G);
        int ohi_idx = __shfl_xor(B.hi_idx, off, G);
        float olo = __shfl_xor(B.lo, off, G);
        int olo_idx = __shfl_xor(B.lo_idx, off, G);
        merge_bounds(B, ohi, ohi_idx, olo, olo_idx);
    }
}

template <int G, int S>
__device__ __forceinline__ void solve_group(const Problem& P, int64_t lp) {
    const int lane = lane_id();
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

    float rx[S], ry[S], rbv[S];
    bool bad = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        int idx = s * G + gl;
        if (idx < m) {
            rx[s] = rax[idx];
            ry[s] = ray[idx];
            rbv[s] = rb[idx];
            bad |= !finite3(rx[s], ry[s], rbv[s]);
        } else {
            rx[s] = 0.0f;
            ry[s] = 0.0f;
            rbv[s] = 0.0f;
        }
    }
    for (int idx = S * G + gl; idx < m; idx += G) bad |= !finite3(rax[idx], ray[idx], rb[idx]);
    bool any_bad = (__ballot(bad) & gmask) != 0;

    LpState st;
    init_state(st, cx, cy);
    if (!ok || any_bad) {
        st.kind = kDead;
        st.dead_status = kInvalid;
    }
    bool done = lp < 0 || st.kind == kDead || m == 0;
    int cur = 0;
    int n1d = 0;

    // one 1D LP on the row violated at index v (held by lane `src` in slot s_v
    // when v < S*G); `s_hi` is the last slot that holds rows below v
    auto run_1dlp = [&](int v, float lx, float ly, float lb, auto slots_static, int s_dyn_end) {
        ++n1d;
        if (lx == 0.0f && ly == 0.0f) {
            st.kind = kDead;
            st.dead_status = kInfeasible;
            return;
        }
        Line L;
        make_line(L, lx, ly, lb);
        Bounds B;
        init_bounds(B);
        constexpr int NS = decltype(slots_static)::value;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            int idx = t * G + gl;
            if (idx < v) work_unit(rx[t], ry[t], rbv[t], idx, L, B);
        }
        for (int t = S; t < s_dyn_end; ++t) {
            int idx = t * G + gl;
            if (idx < v) work_unit(rax[idx], ray[idx], rb[idx], idx, L, B);
        }
        group_reduce<G>(B);
        B.par_inf = (__ballot(B.par_inf) & gmask) != 0;
        apply_1dlp(st, v, L, B, cx, cy, rax, ray, rb);
    };

    // register-resident slots
    [&]<int... Is>(std::integer_sequence<int, Is...>) {
        (
            [&] {
                constexpr int s = Is;
                while (true) {
                    bool act = !done && cur < (s + 1) * G;
                    if (__ballot(act) == 0) break;
                    int idx = s * G + gl;
                    bool viol = act && idx >= cur && idx < m && row_violates(rx[s], ry[s], rbv[s], st);
                    uint64_t bal = __ballot(viol) & gmask;
                    if (act) {
                        if (bal == 0) {
                            cur = (s + 1) * G;
                        } else {
                            int src = __builtin_ctzll(bal);
                            int v = s * G + (src - gbase);
                            float lx = __shfl(rx[s], src);
                            float ly = __shfl(ry[s], src);
                            float lb = __shfl(rbv[s], src);
                            run_1dlp(v, lx, ly, lb, std::integral_constant<int, s + 1>{}, 0);
                            cur = v + 1;
                        }
                        if (cur >= m || st.kind == kDead) done = true;
                    }
                }
            }(),
            ...);
    }(std::make_integer_sequence<int, S>{});

    // rows beyond the registers: read from memory
    for (int s = S; __ballot(!done) != 0; ++s) {
        while (true) {
            bool act = !done && cur < (s + 1) * G;
            if (__ballot(act) == 0) break;
            int idx = s * G + gl;
            bool viol = false;
            float tx = 0.0f, ty = 0.0f, tb = 0.0f;
            if (act && idx >= cur && idx < m) {
                tx = rax[idx];
                ty = ray[idx];
                tb = rb[idx];
                viol = row_violates(tx, ty, tb, st);
            }
            uint64_t bal = __ballot(viol) & gmask;
            if (act) {
                if (bal == 0) {
                    cur = (s + 1) * G;
                } else {
                    int src = __builtin_ctzll(bal);
                    int v = s * G + (src - gbase);
                    float lx = __shfl(tx, src);
                    float ly = __shfl(ty, src);
                    float lb = __shfl(tb, src);
                    run_1dlp(v, lx, ly, lb, std::integral_constant<int, S>{}, s + 1);
                    cur = v + 1;
                }
                if (cur >= m || st.kind == kDead) done = true;
            }
        }
    }

    if (lp >= 0 && gl == 0) finish_lp(P, lp, start, st, n1d);
}

template <int G, int S>
__global__ __launch_bounds__(256) void k_group(Problem P) {
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t q = (int64_t)blockIdx.x * LPS_PER_BLOCK + threadIdx.x / G;
    int64_t lp = -1;
    if (q < P.num_lps) lp = P.order ? (int64_t)P.order[q] : q;
    solve_group<G, S>(P, lp);
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

template <int G, int S>
static hipError_t launch_group_t(const Problem& P, hipStream_t stream) {
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t blocks = (P.num_lps + LPS_PER_BLOCK - 1) / LPS_PER_BLOCK;
    hipLaunchKernelGGL((k_group<G, S>), dim3((unsigned)blocks), dim3(256), 0, stream, P);
    return hipGetLastError();
}

#define RGB_GROUP_CASE(G, S) \
    if (g == G && s == S) return launch_group_t<G, S>(P, stream);

bool group_supported(int g, int s) {
#define RGB_GROUP_SUP(G, S) \
    if (g == G && s == S) return true;
    RGB_GROUP_SHAPES(RGB_GROUP_SUP)
#undef RGB_GROUP_SUP
    return false;
}

hipError_t launch_group(const Problem& P, int g, int s, hipStream_t stream) {
    if (P.num_lps == 0) return hipSuccess;
    RGB_GROUP_SHAPES(RGB_GROUP_CASE)
    return hipErrorInvalidValue;
}

}  // namespace rgb
