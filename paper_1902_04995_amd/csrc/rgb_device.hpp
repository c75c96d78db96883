// Device-side numerics of the batched 2D LP solver (gfx950).
//
// One LP: maximize c.x subject to a_i.x <= b_i (Eq. (1)-(2)), solved with
// Seidel's incremental method (Sec. 2.1).  The bounding rows x <= M, x >= -M
// of Sec. 2.1 are symbolic (M -> infinity), so a state is
//   kCorner  the box corner M*(s_x, s_y): a ray from the origin,
//   kRay     a ray p0 + t*q (t -> infinity) along line l,
//   kPoint   the vertex of lines l and h, kept as the FP32 point p,
//   kDead    infeasible or invalid (final).
// A row that the state violates starts a 1D LP on its line over the earlier
// rows (Eq. (3)-(4)): each earlier row is one work unit (Sec. 3) giving a
// left or right bound on the line.
//
// Arithmetic is FP32 with guards that keep every status decision equal to
// the one a serial FP64 Seidel takes:
//   * signs of 2x2 determinants of inputs (which side a row bounds, whether
//     two rows are parallel, the direction c prefers along a line, ray
//     tests) use Kahan's FMA determinant, whose relative error is below
//     2 ulps, so the sign and an exact zero are always right;
//   * a 1D LP is first run fast: every row's position along the line in
//     FP32, min/max, and a running sum of the positions that turns
//     non-finite when a row is parallel to the line or a position
//     overflows; then a careful FP32 rerun decides parallel rows in FP64
//     (Sec. 2.1: the row either leaves the line whole or empties it), where
//     products of FP32 inputs are exact;
//   * when u_left and u_right (Eq. (3)-(4)) are within FP32 noise of each
//     other, infeasibility is decided in FP64 from the two rows that attain
//     them; when a position overflows FP32, the whole 1D LP is decided by an
//     FP64 pass that compares bounds by cross-multiplication.
// x* is recomputed at the end by Cramer's rule from the defining pair, with
// Kahan determinants (a few ulps per component).  A vertex beyond the FP32
// range makes the LP INVALID.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgb {

constexpr int kOptimal = 0;
constexpr int kInfeasible = 1;
constexpr int kUnbounded = 2;
constexpr int kInvalid = 3;
// Internal status of an LP that a fast kernel left to the FP64 fix-up pass
// (an FP32 overflow in one of its 1D LPs); never returned.
constexpr int kDeferred = 4;

constexpr int kCorner = 0;
constexpr int kRay = 1;
constexpr int kPoint = 2;
constexpr int kDead = 3;

constexpr int kNoIdx = 0x7fffffff;
constexpr int64_t kMaxRows = int64_t(1) << 30;

// Near-tie threshold for u_left vs u_right, relative to the bound magnitudes.
constexpr float kTieRel = 1.0e-4f;

struct Problem {
    const int64_t* offsets;
    const float* ax;
    const float* ay;
    const float* b;
    const float* cx;
    const float* cy;
    float* x_out;
    float* y_out;
    int32_t* status;
    int32_t* n1d;          // optional
    const int32_t* order;  // optional: queue position -> LP id
    int64_t num_lps;
    int64_t num_constraints;
};

// ax*px + ay*py with a sign that is always right and an exact zero
// (Kahan's FMA-based 2x2 determinant).
__device__ __forceinline__ float dot2_exact(float ax, float ay, float px, float py) {
    float w = ay * py;
    float e = __builtin_fmaf(ay, py, -w);
    float f = __builtin_fmaf(ax, px, w);
    return f + e;
}

struct LpState {
    int kind;
    int dead_status;
    float px, py, qx, qy;
    float lx, ly, lb;  // line l of a kRay / kPoint state
    int l;             // row index of line l
    float sig;         // kPoint: position of the vertex along u_l
    bool up;           // kPoint: the vertex is u_right (true) or u_left (false) of line l
};

struct Line {
    float lx, ly, lb;   // a_l, b_l
    float ux, uy;       // direction u = (-a_l.y, a_l.x)
    float p0x, p0y;     // b_l a_l / |a_l|^2
    float pscale;       // |p0| / |u|: the scale of positions along the line
};

__device__ __forceinline__ void init_state(LpState& st, float cx, float cy) {
    st.kind = kCorner;
    st.dead_status = kOptimal;
    st.px = 0.0f;
    st.py = 0.0f;
    st.qx = cx > 0.0f ? 1.0f : -1.0f;
    st.qy = cy > 0.0f ? 1.0f : -1.0f;
    st.lx = st.ly = st.lb = 0.0f;
    st.l = -1;
    st.sig = 0.0f;
    st.up = false;
}

// Does row (ax, ay, b) cut off a kPoint state?  (Sec. 2.1, outcome (2).)
__device__ __forceinline__ bool point_violated(float ax, float ay, float b, float px, float py) {
    return __builtin_fmaf(ax, px, __builtin_fmaf(ay, py, -b)) > 0.0f;
}

// Same test for any live state.
__device__ __forceinline__ bool row_violates(float ax, float ay, float b, const LpState& st) {
    if (st.kind == kPoint) return point_violated(ax, ay, b, st.px, st.py);
    float t = dot2_exact(ax, ay, st.qx, st.qy);
    if (t != 0.0f) return t > 0.0f;
    if (st.kind == kCorner) return b < 0.0f;
    // row parallel to the ray's line: compare a.p0 with b in FP64,
    // a.p0 = b_l (a.a_l) / |a_l|^2.  (The empty asm keeps this rare work in
    // its branch instead of letting it be hoisted out of the scan loop.)
    float lx = st.lx, ly = st.ly, lb = st.lb;
    asm volatile("" : "+v"(lx), "+v"(ly), "+v"(lb));
    double l2 = (double)lx * lx + (double)ly * ly;
    double al = (double)ax * lx + (double)ay * ly;
    return (double)lb * al > (double)b * l2;
}

__device__ __forceinline__ void make_line(Line& L, float lx, float ly, float lb) {
    L.lx = lx;
    L.ly = ly;
    L.lb = lb;
    L.ux = -ly;
    L.uy = lx;
    // p0 = b_l a_l / |a_l|^2 with a reciprocal (1 ulp): p0 only has to lie on
    // the line to rounding, and every kernel computes it the same way
    float k = lb * __builtin_amdgcn_rcpf(__builtin_fmaf(lx, lx, ly * ly));
    L.p0x = k * lx;
    L.p0y = k * ly;
    L.pscale = __builtin_fabsf(k);
}

// Position along u of the intersection of line L with row (ax, ay, b), and
// the side it bounds: D = a.u > 0 bounds from the right (an upper bound on
// the position, Eq. (4)), D < 0 from the left (Eq. (3)), D = 0 is parallel.
// sigma = (b - a.p0) / D.  Every kernel uses this one function, so the same
// row always yields the same bits.
__device__ __forceinline__ float wu_sigma(float ax, float ay, float b, const Line& L, float& D) {
    D = dot2_exact(ax, ay, L.ux, L.uy);
    float r = __builtin_fmaf(-ax, L.p0x, __builtin_fmaf(-ay, L.p0y, b));
    return r * __builtin_amdgcn_rcpf(D);
}

// Parallel row (or zero normal): does it empty line L?  The line lies inside
// the row iff N = b |a_l|^2 - b_l (a.a_l) >= 0; decided in FP64, where the
// products of FP32 inputs are exact.
__device__ __forceinline__ bool parallel_empties(float ax, float ay, float b, const Line& L) {
    double n2 = (double)L.lx * L.lx + (double)L.ly * L.ly;
    double N = (double)b * n2 - (double)L.lb * ((double)ax * L.lx + (double)ay * L.ly);
    return N < 0.0;
}

// IEEE minNum / maxNum as single instructions.  Their operands are always
// results of arithmetic (never signalling NaNs), so none of the quieting the
// compiler adds around fminf / fmaxf is needed; a quiet NaN operand is dropped.
__device__ __forceinline__ float vmin(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmax(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmin3(float a, float b, float c) {
    float r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ float vmax3(float a, float b, float c) {
    float r;
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// One work unit (Sec. 3) as candidates: the row's position if it bounds from
// the right (else hi, the neutral value) and if it bounds from the left (else
// lo).  Rows with D >= 0 count as right bounds; a parallel row (D = 0) gives a
// position r * (1/0) that is infinite or NaN, whatever the sign of its exact
// offset.  `chk` sums the positions, so it ends non-finite exactly when some
// row was parallel to the line or its position overflowed (or the sum did);
// the caller then reruns the 1D LP with the careful passes below, which
// decide those rows exactly.  A non-finite candidate never reaches a bound
// that is used unchecked.
__device__ __forceinline__ void wu_candidates(float ax, float ay, float b, const Line& L, float hi, float lo,
                                              float& th, float& tl, float& chk) {
    float D;
    float sig = wu_sigma(ax, ay, b, L, D);
    bool right = D >= 0.0f;
    th = right ? sig : hi;
    tl = right ? lo : sig;
    chk += sig;
}

// Fold one row into the bounds on line L: hi = min over right bounds
// (u_right), lo = max over left bounds (u_left).
__device__ __forceinline__ void work_unit(float ax, float ay, float b, const Line& L, float& hi, float& lo,
                                          float& chk) {
    float th, tl;
    wu_candidates(ax, ay, b, L, hi, lo, th, tl, chk);
    hi = vmin(hi, th);
    lo = vmax(lo, tl);
}

// Four work units folded with v_min3 / v_max3 (the same bounds as four
// work_unit calls: min and max are exact and order-free).
__device__ __forceinline__ void work_units4(const float (&x)[4], const float (&y)[4], const float (&c)[4], const Line& L,
                                            float& hi, float& lo, float& chk) {
    float th[4], tl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) wu_candidates(x[k], y[k], c[k], L, hi, lo, th[k], tl[k], chk);
    hi = vmin3(vmin3(hi, th[0], th[1]), th[2], th[3]);
    lo = vmax3(vmax3(lo, tl[0], tl[1]), tl[2], tl[3]);
}

// Bounds of a fast pass as they are handed on: hi = -inf when `chk` says a
// row needs the careful rerun (no genuine right bound is -inf).
__device__ __forceinline__ float flag_rerun(float hi, float chk) {
    return __builtin_isfinite(chk) ? hi : -__builtin_huge_valf();
}

// The careful FP32 rerun of a flagged 1D LP: parallel rows are left out of
// the bounds and decided exactly (par); a non-parallel row whose FP32
// position is not finite sets ovf, and the 1D LP is then decided in FP64.
__device__ __forceinline__ void work_unit_exact(float ax, float ay, float b, const Line& L, float& hi, float& lo,
                                                bool& par, bool& ovf) {
    float D;
    float sig = wu_sigma(ax, ay, b, L, D);
    if (D == 0.0f) {
        par |= parallel_empties(ax, ay, b, L);
        return;
    }
    ovf |= !__builtin_isfinite(sig);
    if (D > 0.0f) hi = sig < hi ? sig : hi;
    else lo = sig > lo ? sig : lo;
}

// The 1D LP of Eq. (3)-(4) in FP64, for the rare case FP32 cannot settle (a
// position beyond the FP32 range).  With D_h = a_l x a_h and N_h = b_h |a_l|^2 - b_l (a_l.a_h), row h
// bounds line l at N_h / D_h (times 1/|a_l|^2) from the right if D_h > 0 and
// from the left if D_h < 0; bounds are compared by cross-multiplication and
// ties keep the smaller row index, so the decisions are those of a serial
// FP64 Seidel that evaluates the same expressions.  One side at a time keeps
// the registers this rare path needs to a few.  Parallel rows are not seen
// here: any of them makes the fast pass's position sum non-finite, and the
// careful FP32 rerun has decided them before this pass runs.
struct Bound64 {
    double N, D;  // position N / D; I = its row, -1: none on this side
    int I;
};

// Fold row h into the best bound of one side (right: the smallest position
// among D > 0, left: the largest among D < 0).
template <bool RIGHT>
__device__ __forceinline__ void exact_row(Bound64& e, float lxf, float lyf, float lbf, float axf, float ayf, float bf,
                                          int h) {
    double lx = lxf, ly = lyf, ax = axf, ay = ayf;
    double D = lx * ay - ly * ax;
    if (RIGHT ? !(D > 0.0) : !(D < 0.0)) return;
    double n2 = lx * lx + ly * ly;
    double dot = lx * ax + ly * ay;
    double N = (double)bf * n2 - (double)lbf * dot;
    bool take = e.I < 0 || (RIGHT ? N * e.D < e.N * D : N * e.D > e.N * D);
    if (take) {
        e.N = N;
        e.D = D;
        e.I = h;
    }
}

// Fold another lane's bound o into e (the same rule: strictly better, or
// equal with a smaller row index).
template <bool RIGHT>
__device__ __forceinline__ void exact_merge(Bound64& e, double oN, double oD, int oI) {
    if (oI < 0) return;
    double l = oN * e.D, r = e.N * oD;
    if (e.I < 0 || (RIGHT ? l < r : l > r) || (l == r && oI < e.I)) {
        e.N = oN;
        e.D = oD;
        e.I = oI;
    }
}

// u_left > u_right from the two sides' FP64 bounds.
__device__ __forceinline__ bool exact_empty(const Bound64& hi, const Bound64& lo) {
    return hi.I >= 0 && lo.I >= 0 && lo.N * hi.D < hi.N * lo.D;
}

// The same decision from the two rows that attain u_left and u_right (a near
// tie in FP32): the expressions of exact_row, for those two rows only.
__device__ __forceinline__ bool exact_lo_gt_hi(const Line& L, float lox, float loy, float lob, float hix,
                                               float hiy, float hib) {
    double lx = L.lx, ly = L.ly, lb = L.lb;
    double n2 = lx * lx + ly * ly;
    double Dlo = lx * (double)loy - ly * (double)lox;
    double Dhi = lx * (double)hiy - ly * (double)hix;
    double Nlo = (double)lob * n2 - lb * (lx * (double)lox + ly * (double)loy);
    double Nhi = (double)hib * n2 - lb * (lx * (double)hix + ly * (double)hiy);
    return Nlo * Dhi < Nhi * Dlo;
}

// Does the 1D LP with bounds (lo, hi) on line L look infeasible, and is the
// FP32 answer too close to call?
__device__ __forceinline__ bool near_tie(const Line& L, float hi, float lo) {
    float scale = __builtin_fabsf(hi) + __builtin_fabsf(lo) + L.pscale;
    return __builtin_fabsf(hi - lo) <= kTieRel * scale;
}

// Direction c prefers along u: first non-zero of (c.u, -u.x, -u.y).
__device__ __forceinline__ bool prefers_up(const Line& L, float cx, float cy) {
    float cu = dot2_exact(cx, cy, L.ux, L.uy);
    if (cu != 0.0f) return cu > 0.0f;
    if (L.ly != 0.0f) return L.ly > 0.0f;
    return L.lx < 0.0f;
}

// New state after a feasible 1D LP on line L (row v) whose chosen end sits
// at position sig along u (+-inf: no bound on that side, a ray).  A vertex
// whose FP32 coordinates overflow ends the LP as INVALID: its optimum (or a
// vertex on its way there) lies outside the range FP32 can represent.
__device__ __forceinline__ void move_to(LpState& st, int v, const Line& L, float sig, bool up) {
    st.l = v;
    st.lx = L.lx;
    st.ly = L.ly;
    st.lb = L.lb;
    if (__builtin_isinf(sig)) {
        st.kind = kRay;
        st.px = L.p0x;
        st.py = L.p0y;
        st.qx = up ? L.ux : -L.ux;
        st.qy = up ? L.uy : -L.uy;
    } else {
        st.kind = kPoint;
        st.sig = sig;
        st.up = up;
        st.px = __builtin_fmaf(sig, L.ux, L.p0x);
        st.py = __builtin_fmaf(sig, L.uy, L.p0y);
        st.qx = 0.0f;
        st.qy = 0.0f;
        if (!__builtin_isfinite(st.px) || !__builtin_isfinite(st.py)) {
            st.kind = kDead;
            st.dead_status = kInvalid;
        }
    }
}

__device__ __forceinline__ void move_on_line(LpState& st, int v, const Line& L, float hi, float lo, bool up) {
    move_to(st, v, L, up ? hi : lo, up);
}

__device__ __forceinline__ void set_dead(LpState& st, int status) {
    st.kind = kDead;
    st.dead_status = status;
}

__device__ __forceinline__ bool row_less(float ax1, float ay1, float b1, float ax2, float ay2, float b2) {
    if (ax1 != ax2) return ax1 < ax2;
    if (ay1 != ay2) return ay1 < ay2;
    return b1 < b2;
}

// Final x*, status for one LP and the output store.  For a kPoint state,
// h is the second row through the vertex.
__device__ __forceinline__ void finish_lp(const Problem& P, int64_t lp, int64_t start, const LpState& st, int h,
                                          int n1d) {
    float nan = __builtin_nanf("");
    float x = nan, y = nan;
    int status;
    if (st.kind == kDead) {
        status = st.dead_status;
    } else if (st.kind == kPoint) {
        float a1x = P.ax[start + st.l], a1y = P.ay[start + st.l], b1 = P.b[start + st.l];
        float a2x = P.ax[start + h], a2y = P.ay[start + h], b2 = P.b[start + h];
        if (row_less(a2x, a2y, b2, a1x, a1y, b1)) {
            float t;
            t = a1x; a1x = a2x; a2x = t;
            t = a1y; a1y = a2y; a2y = t;
            t = b1; b1 = b2; b2 = t;
        }
        // Cramer: W = a1 x a2, X = b1 a2.y - b2 a1.y, Y = a1.x b2 - a2.x b1
        float W = dot2_exact(a1x, -a1y, a2y, a2x);
        float X = dot2_exact(b1, -b2, a2y, a1y);
        float Y = dot2_exact(a1x, -a2x, b2, b1);
        x = X / W;
        y = Y / W;
        status = kOptimal;
    } else {
        status = kUnbounded;
    }
    P.x_out[lp] = x;
    P.y_out[lp] = y;
    P.status[lp] = status;
    // the count is that of the method's path; an INVALID LP has none (kernels
    // stop at different rows once they see a non-finite value)
    if (P.n1d) P.n1d[lp] = status == kInvalid ? 0 : n1d;
}

// Row range of LP lp, checked against the row arrays.  Returns false (and
// the LP is INVALID) when the offsets are out of range, decreasing or huge.
__device__ __forceinline__ bool lp_range(const Problem& P, int64_t lp, int64_t& start, int& m) {
    int64_t s = P.offsets[lp], e = P.offsets[lp + 1];
    if (s < 0 || e < s || e > P.num_constraints || e - s > kMaxRows) {
        start = 0;
        m = 0;
        return false;
    }
    start = s;
    m = (int)(e - s);
    return true;
}

__device__ __forceinline__ bool finite3(float a, float b, float c) {
    return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

}  // namespace rgb
