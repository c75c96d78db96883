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

#include <type_traits>

#include "rgb_device.hpp"
#include "rgb_internal.hpp"

namespace rgb {

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

// Butterfly over aligned groups of 2^lg lanes: quad_perm xor 1 and xor 2,
// row half-mirror (8), row mirror (16), swizzle swap 16 (32), then the other
// half of the wave (64).  lg is wave-uniform; it is a constant wherever the
// width is fixed at compile time.  The float steps inside a row are single
// v_min/v_max instructions with a DPP source (bounds are never NaN, so the
// IEEE NaN rules of fmin/fmax do not matter); `s_nop 1` supplies the two
// wait states a DPP read needs after a VALU write of its source.
#define RGB_DPP_FSTEP(NAME, OP, CTRL)                                                                   \
    __device__ __forceinline__ float NAME(float v) {                                                    \
        float r;                                                                                        \
        asm volatile("s_nop 1\n\t" OP " %0, %1, %1 " CTRL " row_mask:0xf bank_mask:0xf bound_ctrl:1"     \
                     : "=v"(r)                                                                          \
                     : "v"(v));                                                                         \
        return r;                                                                                       \
    }
RGB_DPP_FSTEP(min_xor1, "v_min_f32_dpp", "quad_perm:[1,0,3,2]")
RGB_DPP_FSTEP(min_xor2, "v_min_f32_dpp", "quad_perm:[2,3,0,1]")
RGB_DPP_FSTEP(min_hmir, "v_min_f32_dpp", "row_half_mirror")
RGB_DPP_FSTEP(min_mir, "v_min_f32_dpp", "row_mirror")
RGB_DPP_FSTEP(max_xor1, "v_max_f32_dpp", "quad_perm:[1,0,3,2]")
RGB_DPP_FSTEP(max_xor2, "v_max_f32_dpp", "quad_perm:[2,3,0,1]")
RGB_DPP_FSTEP(max_hmir, "v_max_f32_dpp", "row_half_mirror")
RGB_DPP_FSTEP(max_mir, "v_max_f32_dpp", "row_mirror")
#undef RGB_DPP_FSTEP

__device__ __forceinline__ float fmin_(float a, float b) { return b < a ? b : a; }
__device__ __forceinline__ float fmax_(float a, float b) { return b > a ? b : a; }
__device__ __forceinline__ int imin_(int a, int b) { return a < b ? a : b; }

__device__ __forceinline__ float group_min(float v, int lg) {
    if (lg >= 1) v = min_xor1(v);
    if (lg >= 2) v = min_xor2(v);
    if (lg >= 3) v = min_hmir(v);
    if (lg >= 4) v = min_mir(v);
    if (lg >= 5) v = fmin_(v, __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F)));
    if (lg >= 6) v = fmin_(v, __shfl_xor(v, 32));
    return v;
}

__device__ __forceinline__ float group_max(float v, int lg) {
    if (lg >= 1) v = max_xor1(v);
    if (lg >= 2) v = max_xor2(v);
    if (lg >= 3) v = max_hmir(v);
    if (lg >= 4) v = max_mir(v);
    if (lg >= 5) v = fmax_(v, __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F)));
    if (lg >= 6) v = fmax_(v, __shfl_xor(v, 32));
    return v;
}

__device__ __forceinline__ int group_min_i(int v, int lg) {
    if (lg >= 1) v = imin_(v, dpp_i<0xB1>(v));
    if (lg >= 2) v = imin_(v, dpp_i<0x4E>(v));
    if (lg >= 3) v = imin_(v, dpp_i<0x141>(v));
    if (lg >= 4) v = imin_(v, dpp_i<0x140>(v));
    if (lg >= 5) v = imin_(v, __builtin_amdgcn_ds_swizzle(v, 0x401F));
    if (lg >= 6) v = imin_(v, __shfl_xor(v, 32));
    return v;
}

// Compiler-level ordering of LDS accesses between lanes of one wave (the LDS
// executes one wave's instructions in order).
__device__ __forceinline__ void wave_lds_order() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

__device__ __forceinline__ uint64_t group_mask(int lg, int gbase) {
    return lg >= 6 ? ~0ull : (((1ull << (1 << lg)) - 1ull) << gbase);
}

// Rows of one LP, addressed from the batch's (wave-uniform) array bases.
// With WIDE = false the LP's first row is a 32-bit byte offset, so loads use
// the scalar-base + 32-bit vector-offset form and one add per step; batches
// of 2^30 rows or more use 64-bit indices (WIDE = true).
template <bool WIDE>
struct RowRef {
    const float* ax;
    const float* ay;
    const float* b;
    typename std::conditional<WIDE, int64_t, uint32_t>::type first;

    __device__ __forceinline__ float ld(const float* base, int h) const {
        if constexpr (WIDE) {
            return base[first + h];
        } else {
            uint32_t off = (first + (uint32_t)h) * 4u;
            return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + off);
        }
    }
    __device__ __forceinline__ float x(int h) const { return ld(ax, h); }
    __device__ __forceinline__ float y(int h) const { return ld(ay, h); }
    __device__ __forceinline__ float c(int h) const { return ld(b, h); }
};

// The lanes that work on one LP together, as the 1D-LP helpers below see
// them: lane `first()` of `step()` lanes takes rows first(), first() + step(),
// ...; min/max/imin/any combine a value over those lanes and give every one
// of them the result.  GroupLanes is an aligned group of G = 2^lg lanes of a
// wave (DPP butterflies and ballots); the wide kernel's workgroup has its own.
struct GroupLanes {
    int gl, lg;
    uint64_t gmask;
    __device__ __forceinline__ int first() const { return gl; }
    __device__ __forceinline__ int step() const { return 1 << lg; }
    __device__ __forceinline__ float min(float v) const { return group_min(v, lg); }
    __device__ __forceinline__ float max(float v) const { return group_max(v, lg); }
    __device__ __forceinline__ int imin(int v) const { return group_min_i(v, lg); }
    __device__ __forceinline__ bool any(bool b) const { return (__ballot(b) & gmask) != 0; }
};

// Smallest row h < v of the LP whose bound on line L equals `target` on the
// given side; all cooperating lanes must be active.
template <class Rows, class Lanes>
__device__ __forceinline__ int group_find(const Rows& R, int v, const Line& L, float target, bool up,
                                          const Lanes& ln) {
    int best = kNoIdx;
    for (int h = ln.first(); h < v; h += ln.step()) {
        float D;
        float s = wu_sigma(R.x(h), R.y(h), R.c(h), L, D);
        bool hit = (up ? D > 0.0f : D < 0.0f) && s == target;
        best = (hit && h < best) ? h : best;
    }
    return ln.imin(best);
}

// One side of the FP64 1D LP over rows 0 .. v-1 of line L, split over the
// group's lanes and combined with a butterfly of shuffles; every lane gets
// the group's bound.
template <bool RIGHT, class Rows>
__device__ __forceinline__ Bound64 group_exact(const Rows& R, int v, const Line& L, int gl, int lg) {
    Bound64 e{0.0, RIGHT ? 1.0 : -1.0, -1};
    for (int h = gl; h < v; h += (1 << lg)) exact_row<RIGHT>(e, L.lx, L.ly, L.lb, R.x(h), R.y(h), R.c(h), h);
    for (int s = 1; s < (1 << lg); s <<= 1)
        exact_merge<RIGHT>(e, __shfl_xor(e.N, s), __shfl_xor(e.D, s), __shfl_xor(e.I, s));
    return e;
}

// After the fast pass of a 1D LP (bounds known on every cooperating lane;
// hi = -inf flags a parallel or overflowing row): the careful rerun when
// flagged, the exact decision of a near tie from its two bounding rows, then
// the new state.  A position that overflows FP32 needs the FP64 pass over the
// whole 1D LP: with EXACT it runs here (a group of one wave only), otherwise
// the LP is deferred (it stops with the internal status kDeferred and the
// fix-up kernel solves it again with EXACT), which keeps that pass and its
// registers out of the fast kernels.
template <bool EXACT, class Rows, class Lanes>
__device__ __forceinline__ void settle_1dlp(LpState& st, const Rows& R, int v, float hi, float lo, const Line& L,
                                            float cx, float cy, const Lanes& ln) {
    if (hi == -__builtin_huge_valf()) {
        bool par = false, ovf = false;
        hi = __builtin_huge_valf();
        lo = -__builtin_huge_valf();
        for (int h = ln.first(); h < v; h += ln.step()) work_unit_exact(R.x(h), R.y(h), R.c(h), L, hi, lo, par, ovf);
        hi = ln.min(hi);
        lo = ln.max(lo);
        if (ln.any(par)) {
            set_dead(st, kInfeasible);
            return;
        }
        if (ln.any(ovf)) {
            if constexpr (!EXACT) {
                set_dead(st, kDeferred);
            } else {
                const bool up = prefers_up(L, cx, cy);
                const Bound64 eh = group_exact<true>(R, v, L, ln.gl, ln.lg);
                const Bound64 el = group_exact<false>(R, v, L, ln.gl, ln.lg);
                if (exact_empty(eh, el)) {
                    set_dead(st, kInfeasible);
                    return;
                }
                const int k = up ? eh.I : el.I;
                float sig = up ? __builtin_huge_valf() : -__builtin_huge_valf();
                if (k >= 0) {
                    float D;
                    sig = wu_sigma(R.x(k), R.y(k), R.c(k), L, D);
                    if (!__builtin_isfinite(sig)) {  // the vertex lies beyond the FP32 range
                        set_dead(st, kInvalid);
                        return;
                    }
                }
                move_to(st, v, L, sig, up);
            }
            return;
        }
    }
    bool inf = false;
    if (!__builtin_isinf(hi) && !__builtin_isinf(lo)) {
        inf = lo > hi;
        if (near_tie(L, hi, lo)) {
            int il = group_find(R, v, L, lo, false, ln);
            int ih = group_find(R, v, L, hi, true, ln);
            if (il != kNoIdx && ih != kNoIdx)
                inf = exact_lo_gt_hi(L, R.x(il), R.y(il), R.c(il), R.x(ih), R.y(ih), R.c(ih));
        }
    }
    if (inf) set_dead(st, kInfeasible);
    else move_on_line(st, v, L, hi, lo, prefers_up(L, cx, cy));
}

// Where the rows attaining the last 1D LP's bound were seen (kept by the
// cached group path): `mine` has the bit of every lane whose own bound equals
// its group's on that 1D LP, and such a lane's `rec` names the first step of
// its work-unit loops that reached that bound: a row below `from` = min(cs,
// rg) starts a step of the LDS loop, a row below cs a step of the memory loop
// (U rows rec + k G, clamped below those bounds as the loops clamp them), any
// other row is one of the chunk's own rows.  cs is the chunk holding the
// line's row, C rows per chunk.  A group with no bit in `mine` has no record.
struct FindHint {
    uint64_t mine = 0;
    int rec = kNoIdx;
    int C = 1, rg = 0, U = 4;
};

// Smallest row attaining bound st.sig on line L from the record: each lane
// holding the bound tests the rows of its recorded step again (the lane took
// its rows in increasing order and kept the first step that reached its
// bound, so the step holds the lane's smallest attaining row, or a clamped
// repeat of a row no larger than its later ones), and the group takes the
// smallest hit.  Every attaining row's own lane holds the bound, so the
// result is the row group_find would return, from U rows instead of st.l.
template <class Rows>
__device__ __forceinline__ int recorded_find(const Rows& R, const LpState& st, const Line& L, const FindHint& hint,
                                             const GroupLanes& ln) {
    int f = kNoIdx;
    if ((hint.mine >> __lane_id()) & 1ull) {
        const int G = ln.step();
        const int cs = st.l & -hint.C;
        const int from = cs < hint.rg ? cs : hint.rg;
        const bool own = hint.rec >= cs;
        const int bound = hint.rec < from ? from : cs;
        for (int k = 0; k < (own ? 1 : hint.U); ++k) {
            int hk = hint.rec + k * G;
            hk = own || hk < bound ? hk : bound - 1;
            float D;
            const float s = wu_sigma(R.x(hk), R.y(hk), R.c(hk), L, D);
            const bool hit = (st.up ? D > 0.0f : D < 0.0f) && s == st.sig;
            f = hit && hk < f ? hk : f;
        }
    }
    return ln.imin(f);
}

// End of one LP on its group: an LP that died early still gets its remaining
// rows checked for non-finite values, a vertex gets its second defining row
// (from the record when the group has one, else by a pass over the rows below
// its line), and the group's first lane stores the result.
template <bool WIDE>
__device__ __forceinline__ void finish_group(const Problem& P, int64_t lp, int64_t start, const RowRef<WIDE>& R,
                                             LpState& st, int cur, int m, bool bad, int n1d, int gl, int lg,
                                             uint64_t gmask, const FindHint& hint = FindHint{}) {
    if (lp >= 0 && st.kind == kDead && st.dead_status == kInfeasible)
        for (int idx = cur + gl; idx < m; idx += (1 << lg)) bad |= !finite3(R.x(idx), R.y(idx), R.c(idx));
    if ((__ballot(bad) & gmask) != 0) set_dead(st, kInvalid);
    int h = -1;
    if (__ballot(st.kind == kPoint) != 0) {
        if (st.kind == kPoint) {
            Line L;
            make_line(L, R.x(st.l), R.y(st.l), R.c(st.l));
            const GroupLanes ln{gl, lg, gmask};
            h = (hint.mine & gmask) != 0 ? recorded_find(R, st, L, hint, ln) : group_find(R, st.l, L, st.sig, st.up, ln);
            if (h == kNoIdx) h = st.l;  // cannot happen (the bound came from these bits); x is NaN then
        }
    }
    if (lp >= 0 && gl == 0) finish_lp(P, lp, start, st, h, n1d);
}

// ---------------------------------------------------------------------------
// plain: one LP per lane
// ---------------------------------------------------------------------------
// Rows of one LP from its own pointers (one lane walks them serially).
struct PtrRows {
    const float* ax;
    const float* ay;
    const float* b;
    __device__ __forceinline__ float x(int h) const { return ax[h]; }
    __device__ __forceinline__ float y(int h) const { return ay[h]; }
    __device__ __forceinline__ float c(int h) const { return b[h]; }
};

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
    const PtrRows R{P.ax + start, P.ay + start, P.b + start};
    const uint64_t me = 1ull << __lane_id();
    bool bad = false;
    int i = 0;
    for (; i < m && st.kind != kDead; ++i) {
        float ax = R.x(i), ay = R.y(i), b = R.c(i);
        if (!finite3(ax, ay, b)) {
            bad = true;
            break;
        }
        if (!row_violates(ax, ay, b, st)) continue;
        if (ax == 0.0f && ay == 0.0f) {  // 0 <= b with b < 0
            set_dead(st, kInfeasible);
            break;
        }
        ++n1d;
        Line L;
        make_line(L, ax, ay, b);
        float hi = __builtin_huge_valf(), lo = -__builtin_huge_valf(), chk = 0.0f;
        for (int h = 0; h < i; ++h) work_unit(R.x(h), R.y(h), R.c(h), L, hi, lo, chk);
        settle_1dlp<false>(st, R, i, flag_rerun(hi, chk), lo, L, cx, cy, GroupLanes{0, 0, me});
    }
    for (++i; i < m && !bad; ++i) bad = !finite3(R.x(i), R.y(i), R.c(i));
    if (bad) set_dead(st, kInvalid);
    int h = -1;
    if (st.kind == kPoint) {
        Line L;
        make_line(L, R.x(st.l), R.y(st.l), R.c(st.l));
        h = group_find(R, st.l, L, st.sig, st.up, GroupLanes{0, 0, me});
        if (h == kNoIdx) h = st.l;  // cannot happen (the bound came from these bits); x is NaN then
    }
    finish_lp(P, lp, start, st, h, n1d);
}

// Reduce the bounds of a fast 1D-LP pass over the group and settle the 1D LP.
// Only the bound the objective climbs towards is reduced (u_right when c
// prefers +u, otherwise u_left, taken as the minimum of -u_left), with one
// butterfly; whether the other side crosses it or comes within FP32 noise of
// it is decided by one ballot over the lanes' own opposite bounds (the lane
// holding the opposite extreme flags whenever the full test would).  A
// flagged 1D LP, or one whose fast pass needs the careful rerun (a lane's
// position sum is not finite), reduces the other side too and settles as
// settle_1dlp does; every outcome equals the two-sided reduction's.
template <bool EXACT, class Rows>
__device__ __forceinline__ void settle_group(LpState& st, const Rows& R, int v, float hi, float lo, float chk,
                                             const Line& L, float cx, float cy, const GroupLanes& ln) {
    const float ninf = -__builtin_huge_valf();
    const bool up = prefers_up(L, cx, cy);
    const float r = ln.min(__builtin_isfinite(chk) ? (up ? hi : -lo) : ninf);
    const float opp = up ? lo : -hi;
    const bool flag = r == ninf || (!__builtin_isinf(r) && !__builtin_isinf(opp) && (opp > r || near_tie(L, r, opp)));
    if (!ln.any(flag)) {
        move_to(st, v, L, up ? r : -r, up);
        return;
    }
    const float og = ln.max(opp);
    const float hg = r == ninf ? ninf : (up ? r : -og);
    const float lgb = up ? og : -r;
    settle_1dlp<EXACT>(st, R, v, hg, lgb, L, cx, cy, ln);
}

// The rows of one scan chunk a lane holds: rows c0 + gl + k G, k < SR.
template <int SR>
struct Chunk {
    float x[SR], y[SR], c[SR];
};

// Load chunk c0 (m >= 1): rows past the LP's end repeat row m - 1, so every
// load is in range and none needs a branch; they are never tested.
template <int SR, class Rows>
__device__ __forceinline__ void load_chunk(Chunk<SR>& ch, const Rows& R, int c0, int gl, int G, int m) {
#pragma unroll
    for (int k = 0; k < SR; ++k) {
        int idx = c0 + gl + k * G;
        idx = idx < m ? idx : m - 1;
        ch.x[k] = R.x(idx);
        ch.y[k] = R.y(idx);
        ch.c[k] = R.c(idx);
    }
}

// Solve the LP `lp` (-1: none) with a group of G = 2^lg lanes; every lane of
// the wave calls this together, each group with its own LP.  LGC >= 0 fixes
// lg at compile time; LGC = -1 takes it from lg_rt (one body for any width,
// which keeps the persistent kernel's register count at one width's).
//
// The scan (Sec. 2.1, outcome (1) or (2) per row) walks the LP in chunks of
// SR G rows held in registers, SR rows per lane; a chunk's rows are checked
// for non-finite values once, when it arrives.  The first violated row of the
// chunk is found by ballots; after its 1D LP the rest of the same chunk is
// tested again from the registers, so a violation costs no reload.  The 1D LP on
// row v (Eq. (3)-(4)) takes rows below the chunk from memory, U work units
// per lane per step with their loads issued together, and the chunk's own
// rows below v from the registers.
//
// With CACHE > 0 the wave keeps the leading rows of its LPs in LDS (`lds`,
// 3 CACHE floats: x, y and c, each split evenly between the wave's groups,
// so a group keeps its LP's first CACHE G / 64 rows).  The rows are stored
// when their chunk arrives, and 1D LPs read them from LDS: most re-reads fall
// on the leading rows (Seidel's order makes row h's expected re-reads about
// 2 ln(m / h)).  Only the wave's own lanes touch its part of LDS, and the LDS
// executes one wave's accesses in order, so no barrier is needed.
template <int LGC, bool WIDE, bool EXACT = false, int SR = 1, int U = 4, int CACHE = 0, bool TRACK = false>
__device__ __forceinline__ void solve_group(const Problem& P, int64_t lp, int lg_rt = 0, float* lds = nullptr) {
    static_assert(SR >= 1 && U >= 4 && U % 4 == 0, "scan rows and work units per lane");
    static_assert(!TRACK || CACHE > 0, "the record is kept by the cached path");
    const int lg = LGC >= 0 ? LGC : lg_rt;
    const int G = 1 << lg;
    const int C = SR * G;  // rows per chunk
    const int lane = __lane_id();
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const uint64_t gmask = group_mask(lg, gbase);

    int64_t start = 0;
    int m = 0;
    float cx = 0.0f, cy = 0.0f;
    bool ok = false;
    if (lp >= 0) {
        cx = P.cx[lp];
        cy = P.cy[lp];
        ok = lp_range(P, lp, start, m) && __builtin_isfinite(cx) && __builtin_isfinite(cy);
    }
    RowRef<WIDE> R{P.ax, P.ay, P.b, (typename std::conditional<WIDE, int64_t, uint32_t>::type)start};

    LpState st;
    init_state(st, cx, cy);
    if (lp >= 0 && !ok) set_dead(st, kInvalid);
    bool done = lp < 0 || !ok || m == 0;
    int n1d = 0;
    int cs = 0;          // first row of the current chunk
    int pos = 0;         // rows below pos are settled
    bool fresh = true;   // the current chunk has not been checked yet
    Chunk<SR> cur;
    if (!done) load_chunk(cur, R, 0, gl, G, m);
    // this group's rows in LDS: rows [0, rg) of its LP
    const int rg = CACHE >> (6 - lg);
    float* const kx = CACHE ? lds + (lane >> lg) * rg : nullptr;
    float* const ky = CACHE ? kx + CACHE : nullptr;
    float* const kc = CACHE ? kx + 2 * CACHE : nullptr;
    // With TRACK, each 1D LP also records where its bound was reached
    // (FindHint), so the end of the LP needs no pass over the rows below its
    // line.  The record costs a few instructions per work-unit step and a
    // register: it pays on large LPs, whose last line lies thousands of rows
    // in and whose rows are no longer in any cache by the end.
    FindHint hint;
    hint.C = C;
    hint.rg = rg;
    hint.U = U;

    while (__ballot(!done) != 0) {
        if (fresh && !done) {  // a non-finite row anywhere makes the LP INVALID
            bool nf = false;
#pragma unroll
            for (int k = 0; k < SR; ++k) nf |= cs + gl + k * G < m && !finite3(cur.x[k], cur.y[k], cur.c[k]);
            if ((__ballot(nf) & gmask) != 0) {
                set_dead(st, kInvalid);
                done = true;
            }
            if constexpr (CACHE > 0) {
#pragma unroll
                for (int k = 0; k < SR; ++k) {
                    const int idx = cs + gl + k * G;
                    if (idx < rg && idx < m) {
                        kx[idx] = cur.x[k];
                        ky[idx] = cur.y[k];
                        kc[idx] = cur.c[k];
                    }
                }
                wave_lds_order();
            }
        }
        fresh = false;
        // the first violated row at or after pos: the smallest k with a hit,
        // then the group's lowest lane
        uint64_t bal = 0;
        int ksel = 0;
        float sx = 0.0f, sy = 0.0f, sb = 0.0f;
        if (__ballot(!done && st.kind != kPoint) == 0) {  // every live LP of the wave is at a vertex
#pragma unroll
            for (int k = SR - 1; k >= 0; --k) {
                const int idx = cs + gl + k * G;
                const bool viol = !done && idx >= pos && idx < m &&
                                  point_violated(cur.x[k], cur.y[k], cur.c[k], st.px, st.py);
                const uint64_t bk = __ballot(viol) & gmask;
                if (bk != 0) {
                    bal = bk;
                    ksel = k;
                    sx = cur.x[k];
                    sy = cur.y[k];
                    sb = cur.c[k];
                }
            }
        } else {
#pragma unroll
            for (int k = SR - 1; k >= 0; --k) {
                const int idx = cs + gl + k * G;
                const bool viol = !done && idx >= pos && idx < m && row_violates(cur.x[k], cur.y[k], cur.c[k], st);
                const uint64_t bk = __ballot(viol) & gmask;
                if (bk != 0) {
                    bal = bk;
                    ksel = k;
                    sx = cur.x[k];
                    sy = cur.y[k];
                    sb = cur.c[k];
                }
            }
        }
        if (bal == 0) {
            if (!done) {  // next chunk
                cs += C;
                pos = cs;
                if (cs >= m) {
                    done = true;
                } else {
                    load_chunk(cur, R, cs, gl, G, m);
                    fresh = true;
                }
            }
        } else {
            const int src = __builtin_ctzll(bal);
            const int v = cs + ksel * G + (src - gbase);
            float lx, ly, lb;
            if constexpr (LGC == 6) {  // one group per wave: src is wave-uniform
                lx = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, sx), src));
                ly = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, sy), src));
                lb = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, sb), src));
            } else {
                lx = __shfl(sx, src);
                ly = __shfl(sy, src);
                lb = __shfl(sb, src);
            }
            if (lx == 0.0f && ly == 0.0f) {  // 0 <= b with b < 0
                set_dead(st, kInfeasible);
            } else {
                ++n1d;
                Line L;
                make_line(L, lx, ly, lb);
                float hi = __builtin_huge_valf(), lo = -__builtin_huge_valf(), chk = 0.0f;
                // rows below the chunk: the leading ones from LDS, the rest from memory
                int from = 0;
                // the first step at which this lane's bound on the side c
                // climbs towards reached its value (a step's first row)
                const bool up = prefers_up(L, cx, cy);
                int rc = kNoIdx;
                if constexpr (CACHE > 0) {
                    from = cs < rg ? cs : rg;
                    for (int h = gl; h < from; h += U * G) {
                        float x[U], y[U], c[U];
#pragma unroll
                        for (int k = 0; k < U; ++k) {
                            int hk = h + k * G;
                            hk = hk < from ? hk : from - 1;
                            x[k] = kx[hk];
                            y[k] = ky[hk];
                            c[k] = kc[hk];
                        }
                        const float h0 = hi, l0 = lo;
#pragma unroll
                        for (int k = 0; k < U; k += 4)
                            work_units4(*reinterpret_cast<const float(*)[4]>(x + k),
                                        *reinterpret_cast<const float(*)[4]>(y + k),
                                        *reinterpret_cast<const float(*)[4]>(c + k), L, hi, lo, chk);
                        if constexpr (TRACK) rc = (up ? hi < h0 : lo > l0) ? h : rc;
                    }
                    for (int h = from + gl; h < cs; h += U * G) {
                        float x[U], y[U], c[U];
#pragma unroll
                        for (int k = 0; k < U; ++k) {
                            int hk = h + k * G;
                            hk = hk < cs ? hk : cs - 1;
                            x[k] = R.x(hk);
                            y[k] = R.y(hk);
                            c[k] = R.c(hk);
                        }
                        const float h0 = hi, l0 = lo;
#pragma unroll
                        for (int k = 0; k < U; k += 4)
                            work_units4(*reinterpret_cast<const float(*)[4]>(x + k),
                                        *reinterpret_cast<const float(*)[4]>(y + k),
                                        *reinterpret_cast<const float(*)[4]>(c + k), L, hi, lo, chk);
                        if constexpr (TRACK) rc = (up ? hi < h0 : lo > l0) ? h : rc;
                    }
                } else if (cs > 2 * G) {
                    for (int h = gl; h < cs; h += U * G) {
                        float x[U], y[U], c[U];
#pragma unroll
                        for (int k = 0; k < U; ++k) {
                            int hk = h + k * G;
                            if constexpr (SR % U != 0) hk = hk < cs ? hk : cs - 1;
                            x[k] = R.x(hk);
                            y[k] = R.y(hk);
                            c[k] = R.c(hk);
                        }
#pragma unroll
                        for (int k = 0; k < U; k += 4)
                            work_units4(*reinterpret_cast<const float(*)[4]>(x + k),
                                        *reinterpret_cast<const float(*)[4]>(y + k),
                                        *reinterpret_cast<const float(*)[4]>(c + k), L, hi, lo, chk);
                    }
                } else {
                    for (int h = gl; h < cs; h += G) work_unit(R.x(h), R.y(h), R.c(h), L, hi, lo, chk);
                }
                // the chunk's rows below v, from the registers
#pragma unroll
                for (int k = 0; k < SR; ++k) {
                    const int idx = cs + gl + k * G;
                    if (idx < v) {
                        const float h0 = hi, l0 = lo;
                        work_unit(cur.x[k], cur.y[k], cur.c[k], L, hi, lo, chk);
                        if constexpr (TRACK) rc = (up ? hi < h0 : lo > l0) ? idx : rc;
                    }
                }
                settle_group<EXACT>(st, R, v, hi, lo, chk, L, cx, cy, GroupLanes{gl, lg, gmask});
                if constexpr (TRACK) {
                    // a lane holds the bound when the 1D LP ended at a vertex
                    // reached by the fast pass (no lane flagged its sum) and
                    // its own bound is the group's
                    const bool flagged = (__ballot(!__builtin_isfinite(chk)) & gmask) != 0;
                    const bool holds = !flagged && st.kind == kPoint && (up ? hi : -lo) == (up ? st.sig : -st.sig);
                    hint.mine = (hint.mine & ~__ballot(true)) | __ballot(holds);
                    hint.rec = rc;
                }
            }
            pos = v + 1;
            if (pos >= m || st.kind == kDead) done = true;
        }
    }
    // rows of later chunks are checked for non-finite values by finish_group
    finish_group(P, lp, start, R, st, cs + C < m ? cs + C : m, m, false, n1d, gl, lg, gmask, hint);
}

// Scan rows per lane by group width 2^lg: a 64-lane group tests 256 rows per
// chunk, 8- to 32-lane groups two rows per lane, 4-lane groups one (more rows
// per lane cut the scan's instructions per row; small LPs violate too often
// in a chunk for more to pay; measured per width).
constexpr int scan_rows(int lg) { return lg >= 6 ? 4 : lg >= 3 ? 2 : 1; }

// Rows of LP kept in LDS per wave (split between its groups) by the group,
// binned and persistent kernels: 3 x 4 B per row, four waves per workgroup,
// sized so that eight (group) or seven (binned, persistent) workgroups fit
// the 160 KB of a CU.
constexpr int kCacheGroup = 384;
constexpr int kCacheBinned = 448;

// Eight waves per SIMD (at most 64 VGPRs, a few spilled at G >= 16): the
// scan and the work units wait on memory, and more waves hide more of it.
// The group kernel records the 1D-LP bound steps (TRACK of solve_group) when
// its LPs average more than kTrackRows rows and it runs 32 or 64 lanes per
// LP: below, the rows a find re-reads are still cached and the record's
// instructions cost more than the find (measured on MI355X).
constexpr int kTrackRows = 2048;
constexpr int kTrackLg = 5;
constexpr bool kPersistTrack = false;

template <int G, bool WIDE, bool TRACK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_group(Problem P) {
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t q = (int64_t)blockIdx.x * LPS_PER_BLOCK + threadIdx.x / G;
    int64_t lp = -1;
    if (q < P.num_lps) lp = P.order ? (int64_t)P.order[q] : q;
    constexpr int LG = G == 4 ? 2 : G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
    __shared__ float cache[4][kCacheGroup ? 3 * kCacheGroup : 1];
    solve_group<LG, WIDE, false, scan_rows(LG), 4, kCacheGroup, TRACK>(P, lp, 0, cache[threadIdx.x >> 6]);
}

// Fix-up pass after every solve: each wave looks at 64 statuses and solves
// the deferred LPs among them again, one at a time with all 64 lanes and the
// FP64 pass compiled in.  Deferred LPs are rare (near ties, overflow), so
// this is mostly one coalesced read of the statuses.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_fixup(Problem P) {
    const int64_t base = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);
    const int64_t q = base + __lane_id();
    uint64_t todo = __ballot(q < P.num_lps && P.status[q] == kDeferred);
    while (todo != 0) {
        const int k = __builtin_ctzll(todo);
        todo &= todo - 1;
        solve_group<6, WIDE, true>(P, base + k);
    }
}

// ---------------------------------------------------------------------------
// pooled: small scan groups, work units pooled over the whole wave
// ---------------------------------------------------------------------------
// Groups of G = 4..16 lanes scan as in the group kernel, but a group that
// finds a violated row waits until enough of the wave's groups wait too.
// Then one round serves all of them: their work units (Sec. 3) are dealt to
// the 64 lanes in proportion to each 1D LP's length, every lane folds its
// units into running bounds, and the bounds meet in LDS through integer
// min/max atomics on order-preserving keys (exact, like the paper's
// shared-memory atomics).  The settling of the 1D LPs then runs once for all
// waiting groups.  This amortises the fixed cost of a violation over up to
// 16 LPs and keeps every lane busy however uneven the 1D LPs are.

// Float <-> int key with the same order (no NaN ever reaches a bound).
__device__ __forceinline__ int fkey(float f) {
    int k = __builtin_bit_cast(int, f);
    return k ^ ((k >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float funkey(int k) { return __builtin_bit_cast(float, k ^ ((k >> 31) & 0x7fffffff)); }

// One waiting group's 1D LP, as published to the wave.
struct alignas(16) PoolRec {
    int v;             // work units: rows 0 .. v-1 (0: none pooled)
    int L, n;          // lanes L .. L+n-1 serve them
    int hi, lo;        // bounds as keys, combined by atomics
    uint32_t first_lo;  // row offset of the LP
    int32_t first_hi;
    int pad;
    float p0x, p0y, ux, uy;
};

struct PoolLds {
    int slot[64];  // lane -> group whose lanes start there, or -1
    PoolRec g[16];
};

// Inclusive prefix sum over each row of 16 lanes.
__device__ __forceinline__ int row_scan_i(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);
    return x;
}
__device__ __forceinline__ float row_scan_f(float x) {
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x111, 0xF, 0xF, false));
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x112, 0xF, 0xF, false));
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x114, 0xF, 0xF, false));
    x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x118, 0xF, 0xF, false));
    return x;
}

// The pooled work units of one round; all 64 lanes call this together after
// the waiting groups published their records (v > 0 for at least one).
template <bool WIDE>
__device__ __forceinline__ void pool_work_units(const Problem& P, PoolLds& S, int K) {
    const int lane = __lane_id();
    // lanes t < K size the shares: group t gets 1 + floor(v_t (64 - k) / W)
    // lanes, k groups taking part, W = sum of v_t.  The shares add up to at
    // most 64 (the sum of the floors is at most 64 - k; FP32 rounding moves
    // the sum by far less than one).
    int vt = lane < K ? S.g[lane].v : 0;
    float fv = (float)vt;
    float W = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, row_scan_f(fv)), 15));
    int k = __popcll(__ballot(lane < 16 && vt > 0));
    float q = (float)(64 - k) * __builtin_amdgcn_rcpf(W);
    int nt = vt > 0 ? 1 + (int)(fv * q) : 0;
    int incl = row_scan_i(nt);
    int Lt = incl - nt;
    int ntot = __builtin_amdgcn_readlane(incl, 15);
    ntot = ntot < 64 ? ntot : 64;
    if (lane < K && nt > 0 && Lt < 64) {
        S.g[lane].L = Lt;
        S.g[lane].n = nt < 64 - Lt ? nt : 64 - Lt;
        S.slot[Lt] = lane;
    }
    wave_lds_order();
    int s = S.slot[lane];
    uint64_t starts = __ballot(s >= 0);
    if (lane < ntot) {
        // this lane serves the group whose lanes start at the nearest start at or below it
        int p = 63 - __builtin_clzll(starts & (~0ull >> (63 - lane)));
        int g = __shfl(s, p);
        const PoolRec& r = S.g[g];
        int v = r.v, L0 = r.L, n = r.n;
        typename std::conditional<WIDE, int64_t, uint32_t>::type first;
        if constexpr (WIDE) first = (int64_t)(((uint64_t)(uint32_t)r.first_hi << 32) | r.first_lo);
        else first = r.first_lo;
        Line L;
        L.p0x = r.p0x;
        L.p0y = r.p0y;
        L.ux = r.ux;
        L.uy = r.uy;
        RowRef<WIDE> R{P.ax, P.ay, P.b, first};
        // four units per step with their loads issued together; indices past
        // the end repeat row v-1, which cannot change a min or a max
        float hi = __builtin_huge_valf(), lo = -__builtin_huge_valf(), chk = 0.0f;
        for (int h = lane - L0; h < v; h += 4 * n) {
            float x[4], y[4], c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int hk = h + k * n < v ? h + k * n : v - 1;
                x[k] = R.x(hk);
                y[k] = R.y(hk);
                c[k] = R.c(hk);
            }
            work_units4(x, y, c, L, hi, lo, chk);
        }
        hi = flag_rerun(hi, chk);
        if (hi != __builtin_huge_valf())
            __hip_atomic_fetch_min(&S.g[g].hi, fkey(hi), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (lo != -__builtin_huge_valf())
            __hip_atomic_fetch_max(&S.g[g].lo, fkey(lo), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    wave_lds_order();
}

// Solve the LP `lp` (-1: none) with a scan group of G = 2^lg lanes (lg 2..4)
// and pooled 1D LPs; every lane of the wave calls this together, each group
// with its own LP, and S is the wave's own LDS block.  A scan step tests RW
// rows per lane (a window of RW G rows).  Scanning goes on while fewer than
// wait8/8 of the live groups wait (wait8 = 0: serve every violation at once).
template <int LGC, int RW, bool WIDE>
__device__ __forceinline__ void solve_pool(const Problem& P, int64_t lp, int lg_rt, PoolLds& S, int wait8) {
    const int lg = LGC >= 0 ? LGC : lg_rt;
    const int G = 1 << lg;
    const int K = 64 >> lg;
    const int lane = __lane_id();
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const int grp = lane >> lg;
    const uint64_t gmask = group_mask(lg, gbase);

    int64_t start = 0;
    int m = 0;
    float cx = 0.0f, cy = 0.0f;
    bool ok = false;
    if (lp >= 0) {
        cx = P.cx[lp];
        cy = P.cy[lp];
        ok = lp_range(P, lp, start, m) && __builtin_isfinite(cx) && __builtin_isfinite(cy);
    }
    RowRef<WIDE> R{P.ax, P.ay, P.b, (typename std::conditional<WIDE, int64_t, uint32_t>::type)start};

    LpState st;
    init_state(st, cx, cy);
    if (lp >= 0 && !ok) set_dead(st, kInvalid);
    bool done = lp < 0 || !ok || m == 0;
    bool bad = false;
    bool pend = false;  // a violated row waits for the next round
    int cur = 0, v = 0;
    int n1d = 0;
    float vx = 0.0f, vy = 0.0f, vb = 0.0f;  // the waiting violated row

    while (true) {
        while (true) {
            const bool scanning = !done && !pend;
            const int nsc = __popcll(__ballot(scanning));
            const int nwt = __popcll(__ballot(pend));
            if (nsc == 0 || (nwt > 0 && nwt * 8 >= (nsc + nwt) * wait8)) break;
            if (scanning) {
                // window: rows cur + gl + k G, k < RW (cur < m here, so m - 1 is a row)
                float tx[RW], ty[RW], tb[RW];
                bool in[RW];
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    int idx = cur + gl + k * G;
                    in[k] = idx < m;
                    int ld = in[k] ? idx : m - 1;
                    tx[k] = R.x(ld);
                    ty[k] = R.y(ld);
                    tb[k] = R.c(ld);
                }
                bool any_np = false;
#pragma unroll
                for (int k = 0; k < RW; ++k) any_np |= in[k];
                const bool all_point = __ballot(any_np && st.kind != kPoint) == 0;
                uint64_t bsel = 0;
                int ksel = RW;
                float sx = 0.0f, sy = 0.0f, sb = 0.0f;
#pragma unroll
                for (int k = RW - 1; k >= 0; --k) {
                    bool fin = finite3(tx[k], ty[k], tb[k]);
                    bad |= in[k] && !fin;
                    bool viol;
                    if (all_point) viol = in[k] && point_violated(tx[k], ty[k], tb[k], st.px, st.py);
                    else viol = in[k] && fin && row_violates(tx[k], ty[k], tb[k], st);
                    uint64_t bk = __ballot(viol) & gmask;
                    if (bk != 0) {
                        bsel = bk;
                        ksel = k;
                        sx = tx[k];
                        sy = ty[k];
                        sb = tb[k];
                    }
                }
                if (bsel == 0) {
                    cur += RW * G;
                    if (cur >= m) done = true;
                } else {
                    int src = __builtin_ctzll(bsel);
                    v = cur + ksel * G + (src - gbase);
                    vx = __shfl(sx, src);
                    vy = __shfl(sy, src);
                    vb = __shfl(sb, src);
                    pend = true;
                    n1d += (vx != 0.0f || vy != 0.0f) ? 1 : 0;  // a zero normal is no 1D LP
                }
            }
        }
        if (__ballot(pend) == 0) break;

        // one round for every waiting group
        const bool zero = vx == 0.0f && vy == 0.0f;  // 0 <= b with b < 0
        Line L;
        make_line(L, vx, vy, vb);
        const bool part = pend && !zero && v > 0;
        S.slot[lane] = -1;
        if (gl == 0) {
            PoolRec& r = S.g[grp];
            r.v = part ? v : 0;
            r.hi = fkey(__builtin_huge_valf());
            r.lo = fkey(-__builtin_huge_valf());
            if (part) {
                r.first_lo = (uint32_t)R.first;
                r.first_hi = WIDE ? (int32_t)((uint64_t)R.first >> 32) : 0;
                r.p0x = L.p0x;
                r.p0y = L.p0y;
                r.ux = L.ux;
                r.uy = L.uy;
            }
        }
        wave_lds_order();
        if (__ballot(part) != 0) pool_work_units<WIDE>(P, S, K);
        if (pend) {
            if (zero) {
                set_dead(st, kInfeasible);
            } else {
                float hi = funkey(S.g[grp].hi), lo = funkey(S.g[grp].lo);
                settle_1dlp<false>(st, R, v, hi, lo, L, cx, cy, GroupLanes{gl, lg, gmask});
            }
            cur = v + 1;
            if (cur >= m || st.kind == kDead) done = true;
            pend = false;
        }
        wave_lds_order();
    }
    finish_group(P, lp, start, R, st, cur, m, bad, n1d, gl, lg, gmask);
}

// Six waves per SIMD (at most 80 VGPRs).
template <int G, int RW, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_pool(Problem P, int wait8) {
    __shared__ PoolLds pool[4];
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t q = (int64_t)blockIdx.x * LPS_PER_BLOCK + threadIdx.x / G;
    int64_t lp = -1;
    if (q < P.num_lps) lp = P.order ? (int64_t)P.order[q] : q;
    constexpr int LG = G == 4 ? 2 : G == 8 ? 3 : 4;
    solve_pool<LG, RW, WIDE>(P, lp, 0, pool[threadIdx.x >> 6], wait8);
}

// ---------------------------------------------------------------------------
// persistent: size bins + device work queue
// ---------------------------------------------------------------------------
// Size class of an LP with m rows: ceil(log2 m), 0 for m <= 1, capped.
__device__ __forceinline__ int size_class(int m) {
    if (m <= 1) return 0;
    int c = 32 - __builtin_clz((unsigned)(m - 1));
    return c < kClasses ? c : kClasses - 1;
}

// Binning: LPs are split into kBinBlocks contiguous ranges; each block counts
// its LPs per class in LDS, one block turns the counts into queue offsets
// (classes largest first, then block order), and the scatter pass writes the
// queue.  No global atomics, so no contention however skewed the sizes.
__device__ __forceinline__ void bin_range(int64_t n, int64_t& lo, int64_t& hi) {
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    lo = (int64_t)blockIdx.x * per;
    hi = lo + per < n ? lo + per : n;
}

__global__ __launch_bounds__(256) void k_bin(Problem P, Workspace W) {
    __shared__ int hist[kClasses];
    if (threadIdx.x < kClasses) hist[threadIdx.x] = 0;
    __syncthreads();
    int64_t lo, hi;
    bin_range(P.num_lps, lo, hi);
    for (int64_t lp = lo + threadIdx.x; lp < hi; lp += blockDim.x) {
        int64_t start;
        int m;
        lp_range(P, lp, start, m);
        int c = size_class(m);
        W.cls[lp] = (uint8_t)c;
        atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < kClasses) W.blocks[blockIdx.x * kClasses + threadIdx.x] = hist[threadIdx.x];
}

// One block of kBinBlocks threads: thread t owns bin block t.  Inclusive
// Hillis-Steele scan over t for all classes at once, then class bases, then
// the sub-batch table of the queue (a sub-batch is 64/G LPs of one class).
__global__ __launch_bounds__(kBinBlocks) void k_scan(Workspace W, PersistPlan plan) {
    __shared__ int s[2][kClasses][kBinBlocks];
    const int t = threadIdx.x;
    int own[kClasses];
#pragma unroll
    for (int c = 0; c < kClasses; ++c) {
        own[c] = W.blocks[t * kClasses + c];
        s[0][c][t] = own[c];
    }
    __syncthreads();
    int src = 0;
    for (int d = 1; d < kBinBlocks; d <<= 1) {
#pragma unroll
        for (int c = 0; c < kClasses; ++c) s[src ^ 1][c][t] = s[src][c][t] + (t >= d ? s[src][c][t - d] : 0);
        src ^= 1;
        __syncthreads();
    }
    // queue order: the wide classes, then the others, each part largest
    // class first
    int base = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int c = kClasses - 1; c >= 0; --c) {
            if ((plan.log2_lanes[c] == kWideLg) != (pass == 0)) continue;
            int incl = s[src][c][t];
            W.blocks[t * kClasses + c] = base + incl - own[c];
            base += s[src][c][kBinBlocks - 1];
        }
    if (t == 0) {
        QueueHeader* Q = W.q;
        int e = 0, sb = 0, j = 0, nw = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int c = kClasses - 1; c >= 0; --c) {
                const bool wide = plan.log2_lanes[c] == kWideLg;
                if (wide != (pass == 0)) continue;
                int n = s[src][c][kBinBlocks - 1];
                int lg = plan.log2_lanes[c];
                Q->e_start[j] = e;
                Q->e_end[j] = e + n;
                Q->lg[j] = lg;
                if (wide) nw += n;  // no sub-batches: the wide kernel takes them
                else sb += (n + (64 >> lg) - 1) >> (6 - lg);
                Q->sb_end[j] = sb;
                e += n;
                ++j;
            }
        Q->num_sb = sb;
        Q->n_wide = nw;
        Q->wide_head = 0;
        int dyn = (int)(((int64_t)sb * plan.dyn_frac_1024) >> 10);
        Q->dyn_begin = sb - dyn;
        for (int x = 0; x < kQueues; ++x) W.heads[x * kHeadStride] = 0;
    }
}

__global__ __launch_bounds__(256) void k_scatter(Problem P, Workspace W) {
    __shared__ int cur[kClasses];
    if (threadIdx.x < kClasses) cur[threadIdx.x] = W.blocks[blockIdx.x * kClasses + threadIdx.x];
    __syncthreads();
    int64_t lo, hi;
    bin_range(P.num_lps, lo, hi);
    for (int64_t lp = lo + threadIdx.x; lp < hi; lp += blockDim.x) {
        int c = W.cls[lp] & (kClasses - 1);
        int pos = atomicAdd(&cur[c], 1);
        if (pos >= 0 && pos < P.num_lps) W.order[pos] = (int32_t)lp;
    }
}

// Queue position of sub-batch k: its class slot j (queue order).
__device__ __forceinline__ int sub_batch_slot(const QueueHeader& Q, int k) {
    int j = 0;
    while (j < kClasses - 1 && k >= Q.sb_end[j]) ++j;
    return j;
}

// Solve sub-batch k (class slot j) of the queue: 64/G LPs of one class,
// G = 2^lg with lg = Q.lg[j] (fixed at compile time when LGC >= 0).
template <int LGC, bool WIDE, bool TRACK = false>
__device__ __forceinline__ void run_sub_batch(const Problem& P, const Workspace& W, const QueueHeader& Q, int k,
                                              int j, float* lds) {
    const int lg = LGC >= 0 ? LGC : Q.lg[j];
    int sb0 = j ? Q.sb_end[j - 1] : 0;
    int first = Q.e_start[j] + ((k - sb0) << (6 - lg));
    int q = first + (__lane_id() >> lg);
    int64_t lp = q < Q.e_end[j] ? (int64_t)W.order[q] : -1;
    if (lp >= P.num_lps) lp = -1;  // never read outside the batch, whatever the queue holds
    solve_group<LGC, WIDE, false, LGC >= 0 ? scan_rows(LGC) : 1, 4, kCacheBinned, TRACK>(P, lp, lg, lds);
}

// Sub-batch k of the queue with the group width of its class fixed at compile
// time (the same code as the group kernel's for that width), recording the
// bound steps where the slot says so.
template <bool WIDE>
__device__ __forceinline__ void run_sub_batch_any(const Problem& P, const Workspace& W, const QueueHeader& Q, int k,
                                                  float* lds) {
    const int j = sub_batch_slot(Q, k);
    switch (Q.lg[j]) {
        case 2: run_sub_batch<2, WIDE>(P, W, Q, k, j, lds); break;
        case 3: run_sub_batch<3, WIDE>(P, W, Q, k, j, lds); break;
        case 4: run_sub_batch<4, WIDE>(P, W, Q, k, j, lds); break;
        case 5: run_sub_batch<5, WIDE, true>(P, W, Q, k, j, lds); break;
        default: run_sub_batch<6, WIDE, true>(P, W, Q, k, j, lds); break;
    }
}

__device__ __forceinline__ void load_header(QueueHeader& Qs, const Workspace& W) {
    if (threadIdx.x < sizeof(QueueHeader) / 4)
        reinterpret_cast<int*>(&Qs)[threadIdx.x] = reinterpret_cast<const int*>(W.q)[threadIdx.x];
    __syncthreads();
}

// Persistent solve.  Sub-batches [0, dyn_begin) are dealt round-robin to the
// waves of the grid (the queue is sorted largest class first, so every wave
// gets a similar mix); the rest go through the device queue, split into
// kQueues interleaved parts with one head each, so that the pops of one
// XCD's waves (workgroups are spread over the XCDs round-robin) mostly hit
// their own counter.  A wave whose part is drained takes from the others,
// `chunk` sub-batches per pop.  Every wave exits once all parts are drained.
// Seven waves per SIMD (at most 72 VGPRs, nothing spilled): more waves hide
// more of the scan's latency; the grid follows the occupancy the runtime
// reports.
template <bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_persist(Problem P, Workspace W,
                                                                                         PersistPlan plan) {
    __shared__ QueueHeader Qs;
    __shared__ float cache[4][kCacheBinned ? 3 * kCacheBinned : 1];
    float* const lds = cache[threadIdx.x >> 6];
    load_header(Qs, W);
    const QueueHeader& Q = Qs;
    const int waves = (int)(gridDim.x * (blockDim.x >> 6));
    const int wid = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    for (int k = wid; k < Q.dyn_begin; k += waves) run_sub_batch<-1, WIDE, kPersistTrack>(P, W, Q, k, sub_batch_slot(Q, k), lds);
    const int chunk = plan.chunk > 0 ? plan.chunk : 1;
    const int ndyn = Q.num_sb - Q.dyn_begin;
    for (int t = 0; t < kQueues; ++t) {
        const int x = (int)((blockIdx.x + t) % kQueues);
        const int len = ndyn > x ? (ndyn - x + kQueues - 1) / kQueues : 0;  // entries of part x
        while (true) {
            int i0 = 0;
            if (__lane_id() == 0) i0 = atomicAdd(&W.heads[x * kHeadStride], chunk);
            i0 = __builtin_amdgcn_readfirstlane(i0);
            if (i0 >= len) break;
            int i1 = min(i0 + chunk, len);
            for (int i = i0; i < i1; ++i) {
                int k = Q.dyn_begin + x + i * kQueues;
                run_sub_batch<-1, WIDE, kPersistTrack>(P, W, Q, k, sub_batch_slot(Q, k), lds);
            }
        }
    }
}

// Binned, non-persistent: one wave per sub-batch in queue order (largest LPs
// first); the grid is an upper bound and surplus waves exit at once.  The
// hardware dispatcher starts a new wave wherever one finishes.  Seven waves
// per SIMD (at most 72 VGPRs): at eight the widest class's chunk registers
// spill.
template <bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_binned(Problem P, Workspace W) {
    __shared__ QueueHeader Qs;
    __shared__ float cache[4][kCacheBinned ? 3 * kCacheBinned : 1];
    float* const lds = cache[threadIdx.x >> 6];
    load_header(Qs, W);
    const int k = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (k >= Qs.num_sb) return;
    run_sub_batch_any<WIDE>(P, W, Qs, k, lds);
}

// ---------------------------------------------------------------------------
// wide: one workgroup of two waves per LP, its leading rows kept in LDS
// ---------------------------------------------------------------------------
// The multi-wave form of the work-unit scheme (Sec. 3, Fig. NewWork: the work
// units of a 1D LP shared by all threads of a block): 128 lanes scan a chunk
// of 128 kWideRows rows of one LP at once and share each 1D LP's work units.
// As the scan passes them, the LP's first kWideCache rows are stored in LDS,
// so the 1D LPs, which re-read every earlier row (Eq. (3)-(4)), read those
// from LDS instead of the cache hierarchy; Seidel's re-reads fall mostly on
// the leading rows (row h is re-read about 2 ln(m / h) times).  The waves
// combine values through an LDS exchange: each wave posts one record, a
// barrier, and every thread reads all records.  Every wave keeps its own copy
// of the LP state and takes the same decisions on the same exchanged values,
// so the state itself is never exchanged.  The FP64 pass of an overflowing 1D
// LP is left to the fix-up kernel (kDeferred).
//
// Measured on MI355X it is slower than one wave per LP for every size class
// (the exchanges put a barrier on each chunk and each 1D LP of a chain that
// is already latency-bound; more waves per LP and larger chunks were slower
// still), so the tuner only picks it where it wins; the shape kept is the
// fastest one measured.
constexpr int kWideWaves = 2;
constexpr int kWideThreads = 64 * kWideWaves;
constexpr int kWideCache = 1650;  // rows of an LP kept in LDS (19.9 KB: eight workgroups fit a CU)
constexpr int kWideRows = 4;      // rows per lane in a scan chunk

struct WideLds {
    float x[kWideCache], y[kWideCache], c[kWideCache];
    float xc[2][kWideWaves][4];  // exchange records, two sets used in turn
};

// The workgroup as the cooperating lanes of the 1D-LP helpers.  A wave can be
// at most one exchange ahead of another (it cannot pass the next barrier
// alone), so a record set is rewritten only after every wave has read it.
struct WideLanes {
    WideLds* S;
    int t;            // thread in the workgroup
    mutable int par;  // record set of the next exchange (the same in every wave)
    __device__ __forceinline__ int first() const { return t; }
    __device__ __forceinline__ int step() const { return kWideThreads; }
    // post this wave's record (wave-uniform values), wait for every wave's
    __device__ __forceinline__ const float (*post(float a, float b, float c, float d) const)[4] {
        if (__lane_id() == 0) {
            float* p = S->xc[par][t >> 6];
            p[0] = a;
            p[1] = b;
            p[2] = c;
            p[3] = d;
        }
        __syncthreads();
        const float(*r)[4] = S->xc[par];
        par ^= 1;
        return r;
    }
    __device__ __forceinline__ float min(float v) const {
        const float(*r)[4] = post(group_min(v, 6), 0.0f, 0.0f, 0.0f);
        float m = r[0][0];
#pragma unroll
        for (int j = 1; j < kWideWaves; ++j) m = fmin_(m, r[j][0]);
        return m;
    }
    __device__ __forceinline__ float max(float v) const {
        const float(*r)[4] = post(group_max(v, 6), 0.0f, 0.0f, 0.0f);
        float m = r[0][0];
#pragma unroll
        for (int j = 1; j < kWideWaves; ++j) m = fmax_(m, r[j][0]);
        return m;
    }
    __device__ __forceinline__ int imin(int v) const {
        const float(*r)[4] = post(__builtin_bit_cast(float, group_min_i(v, 6)), 0.0f, 0.0f, 0.0f);
        int m = __builtin_bit_cast(int, r[0][0]);
#pragma unroll
        for (int j = 1; j < kWideWaves; ++j) m = imin_(m, __builtin_bit_cast(int, r[j][0]));
        return m;
    }
    __device__ __forceinline__ bool any(bool b) const {
        const float(*r)[4] = post(__ballot(b) != 0 ? 1.0f : 0.0f, 0.0f, 0.0f, 0.0f);
        float m = r[0][0];
#pragma unroll
        for (int j = 1; j < kWideWaves; ++j) m = fmax_(m, r[j][0]);
        return m != 0.0f;
    }
};

// Rows of the LP: the leading kWideCache from LDS, the rest from memory.
template <bool WIDE>
struct WideRows {
    const WideLds* S;
    RowRef<WIDE> G;
    __device__ __forceinline__ float x(int h) const { return h < kWideCache ? S->x[h] : G.x(h); }
    __device__ __forceinline__ float y(int h) const { return h < kWideCache ? S->y[h] : G.y(h); }
    __device__ __forceinline__ float c(int h) const { return h < kWideCache ? S->c[h] : G.c(h); }
};

// Fold rows [lo, hi) of the LP into the bounds on line L, four per thread per
// step with their reads issued together (rows past the end repeat row hi - 1,
// which cannot change a min or a max).
template <class Rows>
__device__ __forceinline__ void wide_units(const Rows& R, int lo, int hi, int t, const Line& L, float& bh, float& bl,
                                           float& chk) {
    for (int h = lo + t; h < hi; h += 4 * kWideThreads) {
        float x[4], y[4], c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int hk = h + k * kWideThreads;
            hk = hk < hi ? hk : hi - 1;
            x[k] = R.x(hk);
            y[k] = R.y(hk);
            c[k] = R.c(hk);
        }
        work_units4(x, y, c, L, bh, bl, chk);
    }
}

// LDS view of rows [0, kWideCache) for the work-unit loop.
struct LdsRows {
    const WideLds* S;
    __device__ __forceinline__ float x(int h) const { return S->x[h]; }
    __device__ __forceinline__ float y(int h) const { return S->y[h]; }
    __device__ __forceinline__ float c(int h) const { return S->c[h]; }
};

// Solve LP `lp` with the whole workgroup (every thread calls this together).
template <bool WIDE, int SR>
__device__ __forceinline__ void solve_wide(const Problem& P, int64_t lp, WideLds& S, const WideLanes& ln) {
    constexpr int C = SR * kWideThreads;  // rows per chunk
    const int t = ln.t;
    const int w = t >> 6;
    int64_t start = 0;
    int m = 0;
    const float cx = P.cx[lp], cy = P.cy[lp];
    const bool ok = lp_range(P, lp, start, m) && __builtin_isfinite(cx) && __builtin_isfinite(cy);
    const RowRef<WIDE> G{P.ax, P.ay, P.b, (typename std::conditional<WIDE, int64_t, uint32_t>::type)start};
    const WideRows<WIDE> R{&S, G};

    LpState st;
    init_state(st, cx, cy);
    if (!ok) set_dead(st, kInvalid);
    bool done = !ok || m == 0;
    int n1d = 0;
    int cs = 0;         // first row of the current chunk
    int pos = 0;        // rows below pos are settled
    bool fresh = true;  // the current chunk has not been checked and stored yet
    Chunk<SR> cur;      // rows cs + t + k 256
    if (!done) load_chunk(cur, G, 0, t, kWideThreads, m);

    while (!done) {
        bool nf = false;
        if (fresh) {  // check the new rows and keep the leading ones in LDS
#pragma unroll
            for (int k = 0; k < SR; ++k) {
                const int idx = cs + t + k * kWideThreads;
                if (idx < m) {
                    nf |= !finite3(cur.x[k], cur.y[k], cur.c[k]);
                    if (idx < kWideCache) {
                        S.x[idx] = cur.x[k];
                        S.y[idx] = cur.y[k];
                        S.c[idx] = cur.c[k];
                    }
                }
            }
        }
        fresh = false;
        // this wave's first violated row at or after pos (rows are ordered by
        // k, then wave, then lane), then the workgroup's through the exchange;
        // a non-finite row anywhere in the chunk posts -1 (INVALID)
        int wv = kNoIdx;
        float wx = 0.0f, wy = 0.0f, wb = 0.0f;
        const bool pt = st.kind == kPoint;
#pragma unroll
        for (int k = 0; k < SR; ++k) {
            const int idx = cs + t + k * kWideThreads;
            const bool viol = idx >= pos && idx < m &&
                              (pt ? point_violated(cur.x[k], cur.y[k], cur.c[k], st.px, st.py)
                                  : row_violates(cur.x[k], cur.y[k], cur.c[k], st));
            const uint64_t b = __ballot(viol);
            if (b != 0 && wv == kNoIdx) {
                const int src = __builtin_ctzll(b);
                wv = cs + k * kWideThreads + w * 64 + src;
                wx = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cur.x[k]), src));
                wy = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cur.y[k]), src));
                wb = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cur.c[k]), src));
            }
        }
        if (__ballot(nf) != 0) wv = -1;
        const float(*r)[4] = ln.post(__builtin_bit_cast(float, wv), wx, wy, wb);
        int v = __builtin_bit_cast(int, r[0][0]), vj = 0;
#pragma unroll
        for (int j = 1; j < kWideWaves; ++j) {
            const int vk = __builtin_bit_cast(int, r[j][0]);
            if (vk < v) {
                v = vk;
                vj = j;
            }
        }
        if (v == -1) {
            set_dead(st, kInvalid);
            done = true;
        } else if (v == kNoIdx) {  // next chunk
            cs += C;
            pos = cs;
            if (cs >= m) {
                done = true;
            } else {
                load_chunk(cur, G, cs, t, kWideThreads, m);
                fresh = true;
            }
        } else {
            const float lx = r[vj][1], ly = r[vj][2], lb = r[vj][3];
            if (lx == 0.0f && ly == 0.0f) {  // 0 <= b with b < 0
                set_dead(st, kInfeasible);
            } else {
                ++n1d;
                Line L;
                make_line(L, lx, ly, lb);
                float hi = __builtin_huge_valf(), lo = -__builtin_huge_valf(), chk = 0.0f;
                const int vl = v < kWideCache ? v : kWideCache;
                wide_units(LdsRows{&S}, 0, vl, t, L, hi, lo, chk);
                if (v > kWideCache) wide_units(G, kWideCache, v, t, L, hi, lo, chk);
                // both sides in one exchange: the bound c climbs towards (as a
                // minimum) and the other one (as a maximum of its negation)
                const bool up = prefers_up(L, cx, cy);
                const float ninf = -__builtin_huge_valf();
                const float sel = __builtin_isfinite(chk) ? (up ? hi : -lo) : ninf;
                const float opp = up ? lo : -hi;
                const float(*e)[4] = ln.post(group_min(sel, 6), group_max(opp, 6), 0.0f, 0.0f);
                float rs = e[0][0], ro = e[0][1];
#pragma unroll
                for (int j = 1; j < kWideWaves; ++j) {
                    rs = fmin_(rs, e[j][0]);
                    ro = fmax_(ro, e[j][1]);
                }
                const float hg = rs == ninf ? ninf : (up ? rs : -ro);
                const float lgb = up ? ro : -rs;
                settle_1dlp<false>(st, R, v, hg, lgb, L, cx, cy, ln);
            }
            pos = v + 1;
            if (pos >= m || st.kind == kDead) done = true;
        }
    }
    // an LP that died infeasible: the rows after the last chunk may still hold
    // a non-finite value (INVALID)
    if (st.kind == kDead && st.dead_status == kInfeasible) {
        bool bad = false;
        for (int idx = (cs + C < m ? cs + C : m) + t; idx < m; idx += kWideThreads)
            bad |= !finite3(G.x(idx), G.y(idx), G.c(idx));
        if (ln.any(bad)) set_dead(st, kInvalid);
    }
    int h = -1;
    if (st.kind == kPoint) {
        Line L;
        make_line(L, R.x(st.l), R.y(st.l), R.c(st.l));
        h = group_find(R, st.l, L, st.sig, st.up, ln);
        if (h == kNoIdx) h = st.l;  // cannot happen (the bound came from these bits); x is NaN then
    }
    if (t == 0) finish_lp(P, lp, start, st, h, n1d);
}

// Entries [0, n_wide) of the queue (the wide classes, largest first), one LP
// per workgroup at a time, taken from the queue's wide head.  The LDS rows
// (20 KB a workgroup) allow eight workgroups per CU.
template <bool WIDE>
__global__ __launch_bounds__(kWideThreads) void k_wide(Problem P, Workspace W) {
    __shared__ WideLds S;
    __shared__ int next;
    const int t = threadIdx.x;
    const int n = W.q->n_wide;
    WideLanes ln{&S, t, 0};
    while (true) {
        if (t == 0) next = atomicAdd(&W.q->wide_head, 1);
        __syncthreads();
        const int q = next;
        __syncthreads();  // everyone has read `next` before it is written again
        if (q >= n) break;
        int64_t lp = W.order[q];
        if (lp < 0 || lp >= P.num_lps) continue;  // never read outside the batch, whatever the queue holds
        solve_wide<WIDE, kWideRows>(P, lp, S, ln);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// 32-bit byte offsets reach every row of the batch?
static bool wide_rows(const Problem& P) { return P.num_constraints >= (int64_t(1) << 30); }

hipError_t launch_fixup(const Problem& P, hipStream_t stream) {
    if (P.num_lps == 0) return hipSuccess;
    Problem F = P;
    F.order = nullptr;
    int64_t blocks = (P.num_lps + 255) / 256;
    if (wide_rows(P)) hipLaunchKernelGGL(k_fixup<true>, dim3((unsigned)blocks), dim3(256), 0, stream, F);
    else hipLaunchKernelGGL(k_fixup<false>, dim3((unsigned)blocks), dim3(256), 0, stream, F);
    return hipGetLastError();
}

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
    // mean rows per LP above kTrackRows: the recording body (32 and 64 lanes)
    constexpr bool kCanTrack = G >= (1 << kTrackLg);
    if (kCanTrack && P.num_constraints > (int64_t)kTrackRows * P.num_lps) {
        if (wide_rows(P)) hipLaunchKernelGGL((k_group<G, true, kCanTrack>), dim3((unsigned)blocks), dim3(256), 0, stream, P);
        else hipLaunchKernelGGL((k_group<G, false, kCanTrack>), dim3((unsigned)blocks), dim3(256), 0, stream, P);
    } else if (wide_rows(P)) {
        hipLaunchKernelGGL((k_group<G, true>), dim3((unsigned)blocks), dim3(256), 0, stream, P);
    } else {
        hipLaunchKernelGGL((k_group<G, false>), dim3((unsigned)blocks), dim3(256), 0, stream, P);
    }
    return hipGetLastError();
}

bool group_supported(int g) {
    return g == 4 || g == 8 || g == 16 || g == 32 || g == 64;
}

hipError_t launch_persistent(const Problem& P, const Workspace& W, const PersistPlan& plan, int grid, int wide_grid,
                             bool binned, hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end) {
    if (P.num_lps == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin, dim3(kBinBlocks), dim3(256), 0, stream, P, W);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kBinBlocks), 0, stream, W, plan);
    hipLaunchKernelGGL(k_scatter, dim3(kBinBlocks), dim3(256), 0, stream, P, W);
    if (ev_begin) (void)hipEventRecord(ev_begin, stream);
    const bool wide = wide_rows(P);
    bool any_wide = false;
    for (int c = 0; c < kClasses; ++c) any_wide |= plan.log2_lanes[c] == kWideLg;
    if (any_wide) {
        if (wide) hipLaunchKernelGGL(k_wide<true>, dim3(wide_grid), dim3(kWideThreads), 0, stream, P, W);
        else hipLaunchKernelGGL(k_wide<false>, dim3(wide_grid), dim3(kWideThreads), 0, stream, P, W);
    }
    if (binned) {
        // at most one sub-batch per LP plus one partial sub-batch per class
        int64_t max_sb = P.num_lps + kClasses;
        int64_t blocks = (max_sb + 3) / 4;
        if (wide) hipLaunchKernelGGL(k_binned<true>, dim3((unsigned)blocks), dim3(256), 0, stream, P, W);
        else hipLaunchKernelGGL(k_binned<false>, dim3((unsigned)blocks), dim3(256), 0, stream, P, W);
    } else {
        if (wide) hipLaunchKernelGGL(k_persist<true>, dim3(grid), dim3(256), 0, stream, P, W, plan);
        else hipLaunchKernelGGL(k_persist<false>, dim3(grid), dim3(256), 0, stream, P, W, plan);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_fixup(P, stream);
    if (ev_end) (void)hipEventRecord(ev_end, stream);
    return e;
}

int wide_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_wide<false>, kWideThreads, 0) != hipSuccess) return 1;
    return n > 0 ? n : 1;
}

int persist_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persist<false>, 256, 0) != hipSuccess) return 1;
    return n > 0 ? n : 1;
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

template <int G, int RW>
static hipError_t launch_pool_t(const Problem& P, int wait8, hipStream_t stream) {
    constexpr int LPS_PER_BLOCK = 256 / G;
    int64_t blocks = (P.num_lps + LPS_PER_BLOCK - 1) / LPS_PER_BLOCK;
    if (wide_rows(P))
        hipLaunchKernelGGL((k_pool<G, RW, true>), dim3((unsigned)blocks), dim3(256), 0, stream, P, wait8);
    else
        hipLaunchKernelGGL((k_pool<G, RW, false>), dim3((unsigned)blocks), dim3(256), 0, stream, P, wait8);
    return hipGetLastError();
}

bool pool_supported(int g, int rows) {
    return (g == 4 || g == 8 || g == 16) && (rows == 1 || rows == 2 || rows == 4);
}

hipError_t launch_pool(const Problem& P, int g, int rows, int wait8, hipStream_t stream) {
    if (P.num_lps == 0) return hipSuccess;
    if (wait8 < 0 || wait8 > 8 || !pool_supported(g, rows)) return hipErrorInvalidValue;
    switch (g * 8 + rows) {
        case 4 * 8 + 1: return launch_pool_t<4, 1>(P, wait8, stream);
        case 4 * 8 + 2: return launch_pool_t<4, 2>(P, wait8, stream);
        case 4 * 8 + 4: return launch_pool_t<4, 4>(P, wait8, stream);
        case 8 * 8 + 1: return launch_pool_t<8, 1>(P, wait8, stream);
        case 8 * 8 + 2: return launch_pool_t<8, 2>(P, wait8, stream);
        case 8 * 8 + 4: return launch_pool_t<8, 4>(P, wait8, stream);
        case 16 * 8 + 1: return launch_pool_t<16, 1>(P, wait8, stream);
        case 16 * 8 + 2: return launch_pool_t<16, 2>(P, wait8, stream);
        default: return launch_pool_t<16, 4>(P, wait8, stream);
    }
}

}  // namespace rgb
