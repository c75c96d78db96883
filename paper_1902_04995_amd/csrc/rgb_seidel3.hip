// Batched three-dimensional LPs by Seidel's incremental method.
//
// The paper solves 2D LPs and names higher dimensions as its next step
// (Sec. 6); the method itself is dimension-recursive (Sec. 2.1): when the
// current optimum violates row i, the new optimum lies on row i's boundary,
// found by an (n-1)-dimensional LP over the rows before i.  Here n = 3:
//
//   3D level  scan the rows in order; a violated plane i starts
//   2D level  an LP on plane i over the rows before i, itself incremental:
//             a violated row h starts
//   1D level  an LP on the line where planes i and h meet, over the rows
//             before h: every row is one work unit (Sec. 3) giving a bound
//             on the line's parameter.
//
// Problem: maximize c.x subject to a_i.x <= b_i and the bounding rows
// |x_k| <= M of Sec. 2.1, with M given by the caller.  The result is the
// lexicographically smallest maximiser (smallest x, then y, then z among the
// maximisers), i.e. the objective is perturbed by -eps e_x - eps^2 e_y -
// eps^3 e_z; every comparison of objective values below breaks ties that way.
//
// The box rows are virtual rows 0..5 ahead of the caller's rows (6.. = rows
// 0..): rows 0..2 are s_k x_k <= M with s_k the sign the perturbed objective
// prefers on axis k (+1 if c_k > 0, else -1), rows 3..5 the opposite faces.
// Rows 0..2 define the starting vertex (M s_x, M s_y, M s_z), and they bound
// every direction the perturbed objective climbs, so each 2D and 1D sub-LP,
// which always includes them, has a finite optimum.
//
// Layout: one group of G = 2^lg lanes per LP (G in 4..64), G LPs' worth of
// groups per 256-lane block.  The group scans G rows at a time and finds the
// first violated one with a ballot; the 1D work units are split over the G
// lanes and reduced with cross-lane shuffles.  Arithmetic is FP64 on FP32
// inputs: products of two inputs are exact, so the cross products that decide
// parallel planes and the direction along a line have exact zeros and signs,
// and for inputs that are small integers every decision is exact.  A new
// vertex is the line's point q/|d|^2 moved by the winning bound along d.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rgb.h"
#include "rgb_dpp.hpp"
#include "rgb_internal.hpp"

namespace rgb3 {

constexpr int kOptimal = 0;
constexpr int kInfeasible = 1;
constexpr int kUnbounded = 2;
constexpr int kInvalid = 3;
constexpr int kNoIdx = 0x7fffffff;
constexpr int kBox = 6;  // virtual box rows ahead of the caller's rows

struct Problem3 {
    const int64_t* offsets;
    const float* ax;
    const float* ay;
    const float* az;
    const float* b;
    const float* cx;
    const float* cy;
    const float* cz;
    float* x_out;
    float* y_out;
    float* z_out;
    int32_t* status;
    int64_t num_lps;
    int64_t num_constraints;
    double M;
};

struct V3 {
    double x, y, z;
};

__device__ __forceinline__ double dot(const V3& a, const V3& b) { return fma(a.x, b.x, fma(a.y, b.y, a.z * b.z)); }
// For two rows of FP32 inputs every product is exact in FP64, so each
// component is rounded once (zero exactly when the rows are parallel).
__device__ __forceinline__ V3 cross(const V3& a, const V3& b) {
    return {fma(a.y, b.z, -(a.z * b.y)), fma(a.z, b.x, -(a.x * b.z)), fma(a.x, b.y, -(a.y * b.x))};
}
__device__ __forceinline__ bool is_zero(const V3& a) { return a.x == 0.0 && a.y == 0.0 && a.z == 0.0; }

struct Row {
    V3 a;
    double b;
};

// Virtual row j of an LP whose caller rows start at `start`.
__device__ __forceinline__ Row row_at(const Problem3& P, int64_t start, int j, const V3& s) {
    Row r;
    if (j >= kBox) {
        const int64_t g = start + (j - kBox);
        r.a = {(double)P.ax[g], (double)P.ay[g], (double)P.az[g]};
        r.b = (double)P.b[g];
    } else {
        const int k = j < 3 ? j : j - 3;
        const double sg = (k == 0 ? s.x : k == 1 ? s.y : s.z) * (j < 3 ? 1.0 : -1.0);
        r.a = {k == 0 ? sg : 0.0, k == 1 ? sg : 0.0, k == 2 ? sg : 0.0};
        r.b = P.M;
    }
    return r;
}

// Does v beat w under the perturbed objective (c.v larger, then x, y, z smaller)?
__device__ __forceinline__ bool lex_better(const V3& c, const V3& v, const V3& w) {
    const double fv = dot(c, v), fw = dot(c, w);
    if (fv != fw) return fv > fw;
    if (v.x != w.x) return v.x < w.x;
    if (v.y != w.y) return v.y < w.y;
    return v.z < w.z;
}

// Does the perturbed objective climb along +d?  First non-zero of
// (c.d, -d.x, -d.y, -d.z).
__device__ __forceinline__ bool prefers_up(const V3& c, const V3& d) {
    const double cd = dot(c, d);
    if (cd != 0.0) return cd > 0.0;
    if (d.x != 0.0) return d.x < 0.0;
    if (d.y != 0.0) return d.y < 0.0;
    return d.z < 0.0;
}

__device__ __forceinline__ bool finite4(float a, float b, float c, float d) {
    return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c) && __builtin_isfinite(d);
}

// Row h parallel to plane i (a_h = lambda a_i, or a_h = 0): on plane i,
// a_h.z is the constant lambda b_i, so the row holds on the whole plane iff
// lambda b_i <= b_h.  With k the largest component of a_i this is
// a_h[k] b_i <= b_h a_i[k] (reversed for a_i[k] < 0): products of two FP32
// inputs, exact in FP64.
__device__ __forceinline__ bool parallel_holds(const Row& Ri, const Row& H) {
    if (is_zero(H.a)) return H.b >= 0.0;
    const double ax = __builtin_fabs(Ri.a.x), ay = __builtin_fabs(Ri.a.y), az = __builtin_fabs(Ri.a.z);
    const int k = ax >= ay && ax >= az ? 0 : ay >= az ? 1 : 2;
    const double aik = k == 0 ? Ri.a.x : k == 1 ? Ri.a.y : Ri.a.z;
    const double ahk = k == 0 ? H.a.x : k == 1 ? H.a.y : H.a.z;
    const double lhs = ahk * Ri.b, rhs = H.b * aik;
    return aik > 0.0 ? lhs <= rhs : lhs >= rhs;
}

using rgbd::group_min_d;
using rgbd::group_min_i;

// A caller row as its four FP32 inputs (broadcast as floats: half the
// cross-lane traffic of doubles).
struct Row4 {
    float x, y, z, b;
};
__device__ __forceinline__ Row to_row(const Row4& f) { return {{(double)f.x, (double)f.y, (double)f.z}, (double)f.b}; }
__device__ __forceinline__ Row4 shfl_row4(const Row4& f, int src) {
    return {__shfl(f.x, src), __shfl(f.y, src), __shfl(f.z, src), __shfl(f.b, src)};
}
__device__ __forceinline__ Row4 load_row4(const Problem3& P, int64_t g) { return {P.ax[g], P.ay[g], P.az[g], P.b[g]}; }

struct State3 {
    V3 x;
    int d0, d1, d2;  // virtual rows of the vertex x
    int status;      // kOptimal while alive
    bool dead;
};

// Optimum over box rows 0..2 restricted to plane i (the 2D LP's start): the
// best of the (up to three) points where plane i meets two of the box planes
// and satisfies the third.  False when there is none (plane i misses the
// region those rows bound, so the LP is infeasible).
__device__ __forceinline__ bool plane_start(const Row& Ri, const V3& c, const V3& s, double M, V3& y, int& e0,
                                            int& e1) {
    bool found = false;
    const double ai[3] = {Ri.a.x, Ri.a.y, Ri.a.z};
    const double sv[3] = {s.x, s.y, s.z};
#pragma unroll
    for (int l = 0; l < 3; ++l) {  // l: the free axis, the other two sit on box faces
        const int j = l == 0 ? 1 : 0, k = l == 2 ? 1 : 2;
        if (ai[l] == 0.0) continue;
        const double num = Ri.b - ai[j] * (M * sv[j]) - ai[k] * (M * sv[k]);
        // s_l * num / a_l <= M, without the division's rounding
        const bool ok = ai[l] > 0.0 ? sv[l] * num <= M * ai[l] : sv[l] * num >= M * ai[l];
        if (!ok) continue;
        double v[3];
        v[j] = M * sv[j];
        v[k] = M * sv[k];
        v[l] = num / ai[l];
        const V3 cand = {v[0], v[1], v[2]};
        if (!found || lex_better(c, cand, y)) {
            found = true;
            y = cand;
            e0 = j;
            e1 = k;
        }
    }
    return found;
}

template <int LG>
__device__ void solve3_group(const Problem3& P, int64_t lp) {
    constexpr int G = 1 << LG;
    const int lane = __lane_id();
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const uint64_t gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << gbase);

    int64_t start = 0;
    int mt = kBox;  // virtual rows
    V3 c = {0.0, 0.0, 0.0};
    bool ok = false;
    if (lp >= 0) {
        const float fcx = P.cx[lp], fcy = P.cy[lp], fcz = P.cz[lp];
        const int64_t s0 = P.offsets[lp], e0 = P.offsets[lp + 1];
        ok = s0 >= 0 && e0 >= s0 && e0 <= P.num_constraints && e0 - s0 <= rgb::kMaxRows &&
             __builtin_isfinite(fcx) && __builtin_isfinite(fcy) && __builtin_isfinite(fcz);
        if (ok) {
            start = s0;
            mt = kBox + (int)(e0 - s0);
        }
        c = {(double)fcx, (double)fcy, (double)fcz};
    }
    const V3 s = {c.x > 0.0 ? 1.0 : -1.0, c.y > 0.0 ? 1.0 : -1.0, c.z > 0.0 ? 1.0 : -1.0};

    State3 st;
    st.x = {P.M * s.x, P.M * s.y, P.M * s.z};
    st.d0 = 0;
    st.d1 = 1;
    st.d2 = 2;
    st.status = ok ? kOptimal : kInvalid;
    st.dead = !ok;
    bool done = lp < 0 || !ok || mt == kBox;
    bool bad = false;
    int cur = kBox;  // rows 3..5 hold at the starting corner

    while (__ballot(!done) != 0) {
        // 3D scan window: rows cur .. cur+G-1 against the vertex x
        const int j = cur + gl;
        const bool in = !done && j < mt;
        Row4 F = {0.0f, 0.0f, 0.0f, 0.0f};
        if (in) F = load_row4(P, start + (j - kBox));
        const bool fin = finite4(F.x, F.y, F.z, F.b);
        bad |= in && !fin;
        const Row R = to_row(F);
        const bool viol = in && fin && dot(R.a, st.x) > R.b;
        const uint64_t bal = __ballot(viol) & gmask;
        if (bal == 0) {
            if (!done) {
                cur += G;
                if (cur >= mt) done = true;
            }
            continue;
        }
        // plane i: the first violated row of this group's window
        const int src = __builtin_ctzll(bal);
        const int i = cur + (src - gbase);
        const Row Ri = to_row(shfl_row4(F, src));
        if (is_zero(Ri.a)) {  // 0 <= b with b < 0
            st.dead = true;
            st.status = kInfeasible;
        } else {
            V3 y;
            int e0 = 0, e1 = 1;
            if (!plane_start(Ri, c, s, P.M, y, e0, e1)) {
                st.dead = true;
                st.status = kInfeasible;
            } else {
                int f0 = i, f1 = e0, f2 = e1;
                int cur2 = 3;  // rows 0..2 made the start; rows 3 .. i-1 follow
                while (cur2 < i) {
                    // 2D scan window on plane i: rows cur2 .. against y
                    const int h = cur2 + gl;
                    const bool in2 = h < i;
                    Row4 Fh = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (in2 && h >= kBox) Fh = load_row4(P, start + (h - kBox));
                    const Row Rh = h >= kBox ? to_row(Fh) : row_at(P, start, h, s);
                    const bool viol2 = in2 && dot(Rh.a, y) > Rh.b;
                    const uint64_t bal2 = __ballot(viol2) & gmask;
                    if (bal2 == 0) {
                        cur2 += G;
                        continue;
                    }
                    const int src2 = __builtin_ctzll(bal2);
                    const int hv = cur2 + (src2 - gbase);
                    // box rows are recomputed, caller rows broadcast as floats
                    const Row4 Fb = shfl_row4(Fh, src2);
                    const Row H = hv >= kBox ? to_row(Fb) : row_at(P, start, hv, s);
                    // line L = plane i ^ plane hv: points q/dd + t d
                    const V3 d = cross(Ri.a, H.a);
                    if (is_zero(d)) {
                        // row hv parallel to plane i (or a zero row): it holds
                        // on the whole plane or nowhere on it, decided exactly
                        // (y's violation may be rounding of a point on it)
                        if (parallel_holds(Ri, H)) {
                            cur2 = hv + 1;
                            continue;
                        }
                        st.dead = true;
                        st.status = kInfeasible;
                        break;
                    }
                    // q = b_i (a_hv x d) - b_hv (a_i x d) = (b_i a_hv - b_hv a_i) x d
                    const double dd = dot(d, d);
                    const V3 e = {fma(Ri.b, H.a.x, -(H.b * Ri.a.x)), fma(Ri.b, H.a.y, -(H.b * Ri.a.y)),
                                  fma(Ri.b, H.a.z, -(H.b * Ri.a.z))};
                    const V3 q = cross(e, d);
                    // 1D LP over rows 0 .. hv-1: row g bounds t by
                    // n_g / (dd s_g) with s_g = a_g.d, n_g = dd b_g - a_g.q;
                    // the positive factor dd is left out of the comparison key.
                    // Only the side the objective climbs towards needs its
                    // row; the other side only needs its extreme value.
                    const bool up = prefers_up(c, d);
                    double hi = __builtin_huge_val(), lo = -__builtin_huge_val();
                    int ib = kNoIdx;
                    bool par = false;
                    for (int g = gl; g < hv; g += G) {
                        const Row Rg = row_at(P, start, g, s);
                        const double sg = dot(Rg.a, d);
                        const double ng = fma(dd, Rg.b, -dot(Rg.a, q));
                        if (sg > 0.0) {
                            const double tau = ng / sg;
                            if (tau < hi) {
                                hi = tau;
                                if (up) ib = g;
                            }
                        } else if (sg < 0.0) {
                            const double tau = ng / sg;
                            if (tau > lo) {
                                lo = tau;
                                if (!up) ib = g;
                            }
                        } else {
                            par |= ng < 0.0;  // parallel to L and excludes it
                        }
                    }
                    // the preferred bound as a minimum over the group (the
                    // left side negated), the smallest row index attaining it,
                    // and infeasibility: a bound of the other side crosses it
                    const double key = up ? hi : -lo;
                    const double kmin = group_min_d<LG>(key);
                    const int gb = group_min_i<LG>(key == kmin ? ib : kNoIdx);
                    const double tau = up ? kmin : -kmin;
                    const bool crosses = up ? lo > tau : hi < tau;
                    if ((__ballot(par || crosses) & gmask) != 0) {
                        st.dead = true;
                        st.status = kInfeasible;
                        break;
                    }
                    if (gb == kNoIdx) {  // unreachable: box rows 0..2 bound the climb
                        st.dead = true;
                        st.status = kInvalid;
                        break;
                    }
                    // the vertex q/dd + (tau/dd) d, tau = n_gb/s_gb
                    const double inv = 1.0 / dd;
                    y = {fma(tau, d.x, q.x) * inv, fma(tau, d.y, q.y) * inv, fma(tau, d.z, q.z) * inv};
                    f1 = hv;
                    f2 = gb;
                    cur2 = hv + 1;
                }
                if (!st.dead) {
                    st.x = y;
                    st.d0 = f0;
                    st.d1 = f1;
                    st.d2 = f2;
                }
            }
        }
        cur = i + 1;
        if (cur >= mt || st.dead) done = true;
    }

    // an LP that died early still has its remaining rows checked for
    // non-finite values (INVALID takes precedence)
    if (lp >= 0 && ok && st.dead)
        for (int j = cur + gl; j < mt; j += G) {
            const int64_t g = start + (j - kBox);
            bad |= !finite4(P.ax[g], P.ay[g], P.az[g], P.b[g]);
        }
    bad = (__ballot(bad) & gmask) != 0;
    if (lp >= 0 && gl == 0) {
        const float nan = __builtin_nanf("");
        int status = bad ? kInvalid : st.status;
        float x = nan, y = nan, z = nan;
        if (status == kOptimal) {
            x = (float)st.x.x;
            y = (float)st.x.y;
            z = (float)st.x.z;
            if (st.d0 < kBox || st.d1 < kBox || st.d2 < kBox) status = kUnbounded;
        }
        P.x_out[lp] = x;
        P.y_out[lp] = y;
        P.z_out[lp] = z;
        P.status[lp] = status;
    }
}

// Five waves per SIMD (at most 96 VGPRs, a few dwords spilled on the rare
// paths) hide more of the dependent FP64 chains than four at 102 VGPRs.
template <int G>
__global__ __launch_bounds__(256, 5) void k_seidel3(Problem3 P) {
    constexpr int LG = G == 4 ? 2 : G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
    const int64_t q = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    solve3_group<LG>(P, q < P.num_lps ? q : -1);
}

}  // namespace rgb3

extern "C" rgb_err_t rgb_solve3_batch(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                                      const float* ax, const float* ay, const float* az, const float* b,
                                      const float* cx, const float* cy, const float* cz, double box, float* x_out,
                                      float* y_out, float* z_out, int32_t* status_out, int32_t lanes_per_lp,
                                      void* stream, void* ev_begin, void* ev_end) {
    if (!ctx || num_lps < 0 || num_constraints < 0) return RGB_ERR_INVALID_ARG;
    // the box must be positive and an FP32 value: x is written in FP32, and an
    // optimum on a face of a larger box would not be
    if (!(box > 0.0) || !(box <= 3.4028234663852886e38)) return RGB_ERR_INVALID_ARG;
    const int G = lanes_per_lp == 0 ? 16 : lanes_per_lp;
    if (G != 4 && G != 8 && G != 16 && G != 32 && G != 64) return RGB_ERR_INVALID_ARG;
    if (num_lps > (int64_t(1) << 31) - 1) return RGB_ERR_TOO_LARGE;
    if (num_lps == 0) return RGB_OK;
    if (!offsets || !cx || !cy || !cz || !x_out || !y_out || !z_out || !status_out) return RGB_ERR_INVALID_ARG;
    if (num_constraints > 0 && (!ax || !ay || !az || !b)) return RGB_ERR_INVALID_ARG;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return RGB_ERR_DEVICE;
    const int dev = rgb::ctx_device(ctx);
    if (dev != prev && hipSetDevice(dev) != hipSuccess) return RGB_ERR_DEVICE;
    rgb3::Problem3 P{offsets, ax, ay, az, b, cx, cy, cz, x_out, y_out, z_out, status_out, num_lps, num_constraints, box};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t blocks = (num_lps * G + 255) / 256;
    if (ev_begin) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(ev_begin), st);
    switch (G) {
        case 4: hipLaunchKernelGGL(rgb3::k_seidel3<4>, dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        case 8: hipLaunchKernelGGL(rgb3::k_seidel3<8>, dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        case 16: hipLaunchKernelGGL(rgb3::k_seidel3<16>, dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        case 32: hipLaunchKernelGGL(rgb3::k_seidel3<32>, dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        default: hipLaunchKernelGGL(rgb3::k_seidel3<64>, dim3((unsigned)blocks), dim3(256), 0, st, P); break;
    }
    const hipError_t e = hipGetLastError();
    if (ev_end) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(ev_end), st);
    if (dev != prev) (void)hipSetDevice(prev);
    return e == hipSuccess ? RGB_OK : RGB_ERR_DEVICE;
}
