// Batched LPs in n dimensions (n = 2..5) by Seidel's incremental method.
//
// The paper solves 2D LPs and names higher dimensions as its next step
// (Sec. 6); the method is recursive in the dimension (Sec. 2.1): when the
// current optimum violates row i, the new optimum lies on row i's boundary and
// is the optimum of an LP of one dimension less over the rows before i.  Here
// the recursion is unrolled at compile time, one level per dimension:
//
//   level n      scan the rows in order against the vertex x;
//   level K < n  on the intersection S of the hyperplanes of the rows that
//                started the levels above, an LP over the rows before the one
//                that started it: its start is the best point of S inside the
//                box faces the objective points at, then a scan of the rows
//                against it, each violated row starting level K - 1;
//   level 2      the same on a plane, written once as x = q + u e + v f, so
//                that each violated row gives its line with a few products;
//   level 1      S is a line p + t d: every earlier row is one work unit
//                (Sec. 3) giving a bound on t, split over the group's lanes
//                and reduced to the bound the objective climbs towards.
//
// Problem: maximize c.x subject to a_i.x <= b_i and the bounding rows
// |x_k| <= M of Sec. 2.1, with M given by the caller.  The result is the
// lexicographically smallest maximiser (the smallest x_1, then x_2, ... among
// the maximisers), i.e. the objective is perturbed by -eps e_1 - eps^2 e_2 -
// ...; every comparison of objective values breaks ties that way.
//
// Virtual rows: 0..n-1 are s_k x_k <= M with s_k the sign the perturbed
// objective prefers on axis k (+1 if c_k > 0, else -1), n..2n-1 the opposite
// faces, 2n.. the caller's rows.  The preferred faces bound every direction
// the perturbed objective climbs, so the LP they cut out of any S has a finite
// optimum, a vertex where dim S of them meet; that vertex starts each level.
//
// Arithmetic: FP64 on the FP32 inputs, with relative tolerances where
// rounding would otherwise decide a degenerate case: a row is violated when
// a.x - b exceeds 1e-11 (sum |a_k x_k| + |b|); a row is parallel to the line
// when |a.d| <= 1e-12 |a|_1 |d|_inf; the objective is flat along the line
// when |c.d| <= 1e-12 |c|_1 |d|_inf; a hyperplane depends on the ones above
// when its pivot after elimination is <= 1e-12 of its 1-norm (then the row,
// violated at a point of S and constant on S, empties S: infeasible); two
// vertices tie when their objective values or coordinates differ by at most
// 1e-12 (|c|_1 |x|_1 + |x|_1 + 1).  A vertex this code accepts therefore
// satisfies every row to within 1e-11 of its scale.
//
// Layout: one group of G = 2^lg lanes per LP (G in 4..64), 256 / G LPs per
// 256-lane block.  The scans test G rows at a time and find the first violated
// one with a ballot; the work units of a line are split over the G lanes and
// reduced with cross-lane moves.  The small linear systems (a subspace's start
// vertices by Cramer's rule, a plane by elimination with pivoting) are solved
// redundantly by every lane of the group.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rgb.h"
#include "rgb_dpp.hpp"
#include "rgb_internal.hpp"

namespace rgbn {

constexpr int kOptimal = 0;
constexpr int kInfeasible = 1;
constexpr int kUnbounded = 2;
constexpr int kInvalid = 3;
constexpr int kAlive = -1;
constexpr int kMaxDim = 5;

constexpr double kTolViol = 1e-11;  // a row's violation, relative to its terms at x
constexpr double kTolPar = 1e-12;   // a row parallel to the line, a dependent hyperplane
constexpr double kTolTie = 1e-12;   // equal objective values or coordinates
constexpr double kTolSing = 1e-14;  // a singular system of start-vertex equations

struct ProblemN {
    const int64_t* offsets;
    const float* a;  // [n][num_constraints]
    const float* b;
    const float* c;  // [n][num_lps]
    float* x_out;    // [n][num_lps]
    int32_t* status;
    int64_t num_lps;
    int64_t num_constraints;
    double M;
};

template <int D>
struct Row {
    double a[D];
    double b;
};

constexpr int popc(int v) {
    int n = 0;
    for (; v; v >>= 1) n += v & 1;
    return n;
}

// The set bits of Mask in increasing order (compile-time table).
template <int Mask, int N>
struct Bits {
    int v[N > 0 ? N : 1];
    constexpr Bits() : v() {
        int t = 0;
        for (int k = 0; k < 32 && t < N; ++k)
            if ((Mask >> k) & 1) v[t++] = k;
    }
};

// Cramer's rule for R <= 3 unknowns; false when |det| is at most kTolSing
// times the product of the rows' 1-norms (no single point).
template <int R>
__device__ __forceinline__ bool solve_small(const double (&A)[R][R], const double (&r)[R], double norms,
                                            double (&v)[R]) {
    static_assert(R >= 1 && R <= 3, "start vertices need at most three unknowns");
    if constexpr (R == 1) {
        if (!(__builtin_fabs(A[0][0]) > kTolSing * norms)) return false;
        v[0] = r[0] / A[0][0];
    } else if constexpr (R == 2) {
        const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        if (!(__builtin_fabs(det) > kTolSing * norms)) return false;
        const double inv = 1.0 / det;
        v[0] = (r[0] * A[1][1] - A[0][1] * r[1]) * inv;
        v[1] = (A[0][0] * r[1] - r[0] * A[1][0]) * inv;
    } else {
        auto det3 = [](double a0, double a1, double a2, double b0, double b1, double b2, double c0, double c1,
                       double c2) { return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0); };
        const double det = det3(A[0][0], A[0][1], A[0][2], A[1][0], A[1][1], A[1][2], A[2][0], A[2][1], A[2][2]);
        if (!(__builtin_fabs(det) > kTolSing * norms)) return false;
        const double inv = 1.0 / det;
        v[0] = det3(r[0], A[0][1], A[0][2], r[1], A[1][1], A[1][2], r[2], A[2][1], A[2][2]) * inv;
        v[1] = det3(A[0][0], r[0], A[0][2], A[1][0], r[1], A[1][2], A[2][0], r[2], A[2][2]) * inv;
        v[2] = det3(A[0][0], A[0][1], r[0], A[1][0], A[1][1], r[1], A[2][0], A[2][1], r[2]) * inv;
    }
    return true;
}

template <int D, int LG>
struct Group {
    static constexpr int G = 1 << LG;
    ProblemN P;
    int64_t start;
    int mt;     // virtual rows: the 2D box faces, then the LP's rows
    int smask;  // bit k: the objective prefers +x_k
    int gl, gbase;
    uint64_t gmask;
    double c[D];
    double cn;    // |c|_1
    double x[D];  // the current vertex
    int H[D];     // rows whose hyperplanes define the current subspace
    int status;   // kAlive while the LP is being solved

    __device__ __forceinline__ double sgn(int k) const { return ((smask >> k) & 1) ? 1.0 : -1.0; }

    __device__ __forceinline__ Row<D> row(int j) const {
        Row<D> r;
        if (j >= 2 * D) {
            const int64_t g = start + (j - 2 * D);
#pragma unroll
            for (int k = 0; k < D; ++k) r.a[k] = (double)P.a[k * P.num_constraints + g];
            r.b = (double)P.b[g];
        } else {
            const int k0 = j < D ? j : j - D;
            const bool plus = (((smask >> k0) & 1) != 0) != (j >= D);
#pragma unroll
            for (int k = 0; k < D; ++k) r.a[k] = k == k0 ? (plus ? 1.0 : -1.0) : 0.0;
            r.b = P.M;
        }
        return r;
    }

    static __device__ __forceinline__ bool violates(const Row<D>& r, const double (&v)[D]) {
        double lhs = 0.0, mag = __builtin_fabs(r.b);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = r.a[k] * v[k];
            lhs += t;
            mag += __builtin_fabs(t);
        }
        return lhs - r.b > kTolViol * mag;
    }

    // Does v (objective value fv) beat w (fw) under the perturbed objective:
    // c.v larger, then x_1, x_2, ... smaller?
    __device__ __forceinline__ bool better(const double (&v)[D], double fv, const double (&w)[D], double fw) const {
        double vn = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) vn += __builtin_fabs(v[k]);
        const double tol = kTolTie * (cn * vn + vn + 1.0);
        if (fv > fw + tol) return true;
        if (fv < fw - tol) return false;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (v[k] < w[k] - tol) return true;
            if (v[k] > w[k] + tol) return false;
        }
        return false;
    }
    __device__ __forceinline__ double objective(const double (&v)[D]) const {
        double f = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) f += c[k] * v[k];
        return f;
    }

    // Does the perturbed objective climb along +d?  The sign of c.d unless
    // it is within 1e-12 |c|_1 |d|_inf of zero, else of the first -d_k above
    // 1e-12 |d|_inf.  (Scales are norms, not the products' magnitudes: a
    // component of d that is zero up to rounding must not decide.)
    __device__ __forceinline__ bool prefers_up(const double (&d)[D], double dmax) const {
        double cd = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) cd += c[k] * d[k];
        const double mag = cn * dmax;
        if (cd > kTolTie * mag) return true;
        if (cd < -kTolTie * mag) return false;
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (__builtin_fabs(d[k]) > kTolPar * dmax) return d[k] < 0.0;
        return false;
    }

    // One candidate start vertex of the subspace cut by the R hyperplanes
    // H[0..R): the preferred faces of the axes in Q are tight, the other R
    // coordinates solve the hyperplane equations.  Kept if it lies inside
    // the remaining preferred faces and beats the best so far.
    template <int R, int Q>
    __device__ __forceinline__ void try_start(const Row<D> (&h)[R], double (&best)[D], double& fbest,
                                              bool& found) const {
        constexpr int kU = ((1 << D) - 1) & ~Q;
        constexpr Bits<kU, R> u{};
        double A[R][R], rhs[R];
        double norms = 1.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            double r = h[i].b, nrm = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k)
                if ((Q >> k) & 1) r -= h[i].a[k] * (sgn(k) * P.M);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                A[i][t] = h[i].a[u.v[t]];
                nrm += __builtin_fabs(A[i][t]);
            }
            rhs[i] = r;
            norms *= nrm;
        }
        double v[R];
        if (!solve_small<R>(A, rhs, norms, v)) return;
        double cand[D];
#pragma unroll
        for (int k = 0; k < D; ++k) cand[k] = sgn(k) * P.M;
#pragma unroll
        for (int t = 0; t < R; ++t) cand[u.v[t]] = v[t];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int k = u.v[t];
            if (sgn(k) * cand[k] - P.M > kTolViol * (__builtin_fabs(cand[k]) + P.M)) return;
        }
        const double fc = objective(cand);
        if (!found || better(cand, fc, best, fbest)) {
            found = true;
            fbest = fc;
#pragma unroll
            for (int k = 0; k < D; ++k) best[k] = cand[k];
        }
    }

    template <int R, int Q>
    __device__ __forceinline__ void each_start(const Row<D> (&h)[R], double (&best)[D], double& fbest,
                                               bool& found) const {
        if constexpr (Q < (1 << D)) {
            if constexpr (popc(Q) == D - R) try_start<R, Q>(h, best, fbest, found);
            each_start<R, Q + 1>(h, best, fbest, found);
        }
    }

    // The best point of the subspace cut by H[0..R) inside the preferred
    // faces (the start of its LP); false when there is none (the subspace
    // misses the region those faces bound, so the LP is infeasible).
    template <int R>
    __device__ __forceinline__ bool subspace_start(double (&y)[D]) const {
        Row<D> h[R];
#pragma unroll
        for (int i = 0; i < R; ++i) h[i] = row(H[i]);
        bool found = false;
        double fbest = 0.0;
        each_start<R, 0>(h, y, fbest, found);
        return found;
    }

    // The plane cut by the D - 2 hyperplanes H[0..D-2), as x = q + u e + v f,
    // by elimination with the largest pivot of each row; the two columns
    // never chosen are u and v (e has 1 in the first, 0 in the second, f the
    // reverse).  False when a hyperplane depends on the ones before it.
    __device__ __forceinline__ bool plane(double (&q)[D], double (&e)[D], double (&f)[D]) const {
        constexpr int R = D - 2;
        if constexpr (R == 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                q[k] = 0.0;
                e[k] = k == 0 ? 1.0 : 0.0;
                f[k] = k == 1 ? 1.0 : 0.0;
            }
            return true;
        } else {
            double A[R][D + 1], nrm[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const Row<D> h = row(H[i]);
                nrm[i] = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    A[i][k] = h.a[k];
                    nrm[i] += __builtin_fabs(h.a[k]);
                }
                A[i][D] = h.b;
            }
            int used = 0, pc[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                double best = -1.0, piv = 0.0;
                int bk = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double v = __builtin_fabs(A[i][k]);
                    if (!((used >> k) & 1) && v > best) {
                        best = v;
                        bk = k;
                        piv = A[i][k];
                    }
                }
                if (!(best > kTolPar * nrm[i])) return false;
                pc[i] = bk;
                used |= 1 << bk;
                const double inv = 1.0 / piv;
#pragma unroll
                for (int k = 0; k <= D; ++k) A[i][k] = k == bk ? 1.0 : A[i][k] * inv;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r == i) continue;
                    double g = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        if (k == bk) g = A[r][k];
#pragma unroll
                    for (int k = 0; k <= D; ++k) A[r][k] = k == bk ? 0.0 : __builtin_fma(-g, A[i][k], A[r][k]);
                }
            }
            const int free = ~used & ((1 << D) - 1);
            const int c1 = __builtin_ctz(free), c2 = __builtin_ctz(free & (free - 1));
#pragma unroll
            for (int k = 0; k < D; ++k) {
                q[k] = 0.0;
                e[k] = k == c1 ? 1.0 : 0.0;
                f[k] = k == c2 ? 1.0 : 0.0;
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                double a1 = 0.0, a2 = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    if (k == c1) a1 = A[i][k];
                    if (k == c2) a2 = A[i][k];
                }
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k == pc[i]) {
                        q[k] = A[i][D];
                        e[k] = -a1;
                        f[k] = -a2;
                    }
            }
            return true;
        }
    }

    // The best point of the plane q + u e + v f inside the preferred faces
    // (the start of the plane's LP): where two of the faces meet, inside the
    // others, best by the perturbed objective.  False when there is none.
    __device__ __forceinline__ bool plane_start(const double (&q)[D], const double (&e)[D], const double (&f)[D],
                                                double (&best)[D]) const {
        bool found = false;
        double fbest = 0.0;
#pragma unroll
        for (int k1 = 0; k1 < D; ++k1)
#pragma unroll
            for (int k2 = k1 + 1; k2 < D; ++k2) {
                const double det = e[k1] * f[k2] - f[k1] * e[k2];
                const double sc = (__builtin_fabs(e[k1]) + __builtin_fabs(f[k1])) *
                                  (__builtin_fabs(e[k2]) + __builtin_fabs(f[k2]));
                if (!(__builtin_fabs(det) > kTolSing * sc)) continue;
                const double r1 = sgn(k1) * P.M - q[k1], r2 = sgn(k2) * P.M - q[k2];
                const double inv = 1.0 / det;
                const double u = (r1 * f[k2] - f[k1] * r2) * inv, v = (e[k1] * r2 - r1 * e[k2]) * inv;
                double cand[D];
                bool inside = true;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    cand[k] = k == k1 || k == k2 ? sgn(k) * P.M : __builtin_fma(v, f[k], __builtin_fma(u, e[k], q[k]));
                    if (k != k1 && k != k2)
                        inside = inside && !(sgn(k) * cand[k] - P.M > kTolViol * (__builtin_fabs(cand[k]) + P.M));
                }
                if (!inside) continue;
                const double fc = objective(cand);
                if (!found || better(cand, fc, best, fbest)) {
                    found = true;
                    fbest = fc;
#pragma unroll
                    for (int k = 0; k < D; ++k) best[k] = cand[k];
                }
            }
        return found;
    }

    // The line where row h's hyperplane meets the plane q + u e + v f, as
    // p + t d: with alpha = a.e, beta = a.f, gamma = b - a.q the line is
    // alpha u + beta v = gamma, solved for the variable with the larger
    // coefficient.  False when the row is parallel to the plane (its normal
    // depends on the plane's hyperplanes).
    __device__ __forceinline__ bool line_in_plane(const double (&q)[D], const double (&e)[D], const double (&f)[D],
                                                  const Row<D>& h, double (&p)[D], double (&d)[D]) const {
        double al = 0.0, be = 0.0, aq = 0.0, an = 0.0, bmax = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            al += h.a[k] * e[k];
            be += h.a[k] * f[k];
            aq += h.a[k] * q[k];
            an += __builtin_fabs(h.a[k]);
            bmax = __builtin_fmax(bmax, __builtin_fmax(__builtin_fabs(e[k]), __builtin_fabs(f[k])));
        }
        const double ga = h.b - aq;
        const bool ue = __builtin_fabs(al) >= __builtin_fabs(be);
        const double piv = ue ? al : be, oth = ue ? be : al;
        if (!(__builtin_fabs(piv) > kTolPar * an * bmax)) return false;
        const double r = 1.0 / piv, t0 = ga * r, w = oth * r;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double pv = ue ? e[k] : f[k], ov = ue ? f[k] : e[k];
            p[k] = __builtin_fma(t0, pv, q[k]);
            d[k] = __builtin_fma(-w, pv, ov);
        }
        return true;
    }

    // Level 2: on the plane q + u e + v f (x its start), scan the virtual rows
    // [first, lim) against x; each violated row starts the 1D LP on the line
    // where it meets the plane, over the rows before it.
    __device__ void scan_plane(const double (&q)[D], const double (&e)[D], const double (&f)[D], int first,
                               int lim) {
        int cur = first;
        while (cur < lim) {
            const int j = cur + gl;
            Row<D> r = row(j < lim ? j : 0);
            const bool viol = j < lim && violates(r, x);
            const uint64_t bal = __ballot(viol) & gmask;
            if (bal == 0) {
                cur += G;
                continue;
            }
            const int src = __builtin_ctzll(bal);
            const int hv = cur + (src - gbase);
            // the violated row, from the lane that tested it
#pragma unroll
            for (int k = 0; k < D; ++k) r.a[k] = __shfl(r.a[k], src);
            r.b = __shfl(r.b, src);
            double p[D], d[D];
            if (!line_in_plane(q, e, f, r, p, d)) {
                status = kInfeasible;
                return;
            }
            lp1(p, d, hv);
            if (status != kAlive) return;
            cur = hv + 1;
        }
    }

    // The 1D LP on p + t d over the virtual rows [0, lim): each lane keeps
    // the tightest bound of each side over its rows (for the side the
    // objective does not climb towards, with that row's s = a.d, n = b - a.p
    // and scales); the climbing side's bound is reduced over the group;
    // infeasible when a row parallel to the line excludes it or the other
    // side's tightest row is violated at the new vertex (its residual there
    // is s tau - n).  On success x is that vertex.
    __device__ void lp1(const double (&p)[D], const double (&d)[D], int lim) {
        double dmax = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) dmax = __builtin_fmax(dmax, __builtin_fabs(d[k]));
        const bool up = prefers_up(d, dmax);
        double best = __builtin_huge_val(), other = -__builtin_huge_val();  // in the climbing direction
        double os = 0.0, on = 0.0, oan = 0.0, oapa = 0.0;
        bool par = false;
        for (int g = gl; g < lim; g += G) {
            const Row<D> r = row(g);
            double sv = 0.0, an = 0.0, ap = 0.0, apa = __builtin_fabs(r.b);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                sv += r.a[k] * d[k];
                an += __builtin_fabs(r.a[k]);
                const double q = r.a[k] * p[k];
                ap += q;
                apa += __builtin_fabs(q);
            }
            const double tol = kTolPar * an * dmax;
            const double n = r.b - ap;
            if (sv > tol || sv < -tol) {
                const double t = n / sv;
                // in the climbing direction: a bound ahead (s > 0 when up)
                // caps the climb, a bound behind is the other side
                const bool ahead = (sv > 0.0) == up;
                const double tc = up ? t : -t;
                if (ahead) {
                    best = __builtin_fmin(best, tc);
                } else if (tc > other) {
                    other = tc;
                    os = sv;
                    on = n;
                    oan = an;
                    oapa = apa;
                }
            } else {
                par |= n < -kTolViol * apa;
            }
        }
        const double kmin = rgbd::group_min_d<LG>(best);
        if (!(kmin < __builtin_huge_val())) {  // unreachable: the preferred faces bound the climb
            status = kInvalid;
            return;
        }
        const double tau = up ? kmin : -kmin;
        const bool crosses = other > kmin &&
                             __builtin_fma(os, tau, -on) > kTolViol * (oapa + __builtin_fabs(tau) * oan * dmax);
        if ((__ballot(par || crosses) & gmask) != 0) {
            status = kInfeasible;
            return;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = __builtin_fma(tau, d[k], p[k]);
    }

    template <int K>
    __device__ void descend(int hv);

    // Level K (the current subspace has dimension K, 3 <= K < D): scan the
    // virtual rows [first, lim) against x; each violated row starts level
    // K - 1 on its hyperplane.
    template <int K>
    __device__ void scan(int first, int lim) {
        int cur = first;
        while (cur < lim) {
            const int j = cur + gl;
            bool viol = false;
            if (j < lim) viol = violates(row(j), x);
            const uint64_t bal = __ballot(viol) & gmask;
            if (bal == 0) {
                cur += G;
                continue;
            }
            const int hv = cur + (__builtin_ctzll(bal) - gbase);
            descend<K>(hv);
            if (status != kAlive) return;
            cur = hv + 1;
        }
    }
};

// Row hv, violated at level K, starts level K - 1 on its hyperplane over the
// rows before it.
template <int D, int LG>
template <int K>
__device__ void Group<D, LG>::descend(int hv) {
    H[D - K] = hv;
    if constexpr (K == 2) {  // D == 2: the plane is the whole space
        double q[D], e[D], f[D], p[D], d[D];
        plane(q, e, f);
        if (!line_in_plane(q, e, f, row(hv), p, d)) {
            status = kInfeasible;
            return;
        }
        lp1(p, d, hv);
    } else if constexpr (K == 3) {
        double q[D], e[D], f[D];
        if (!plane(q, e, f)) {
            status = kInfeasible;
            return;
        }
        double y[D];
        if (!plane_start(q, e, f, y)) {
            status = kInfeasible;
            return;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = y[k];
        scan_plane(q, e, f, D, hv);
    } else {
        double y[D];
        if (!subspace_start<D - K + 1>(y)) {
            status = kInfeasible;
            return;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = y[k];
        scan<K - 1>(D, hv);
    }
}

template <int D, int LG>
__device__ void solve_group(const ProblemN& P, int64_t lp) {
    constexpr int G = 1 << LG;
    Group<D, LG> S;
    S.P = P;
    const int lane = __lane_id();
    S.gl = lane & (G - 1);
    S.gbase = lane & ~(G - 1);
    S.gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << S.gbase);
    S.start = 0;
    S.mt = 2 * D;
    S.smask = 0;
    bool ok = false;
    if (lp >= 0) {
        const int64_t s0 = P.offsets[lp], e0 = P.offsets[lp + 1];
        ok = s0 >= 0 && e0 >= s0 && e0 <= P.num_constraints && e0 - s0 <= rgb::kMaxRows;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float ck = P.c[k * P.num_lps + lp];
            ok = ok && __builtin_isfinite(ck);
            S.c[k] = (double)ck;
            if (ck > 0.0f) S.smask |= 1 << k;
        }
        if (ok) {
            S.start = s0;
            S.mt = 2 * D + (int)(e0 - s0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) S.c[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        S.x[k] = S.sgn(k) * P.M;
        S.H[k] = 0;
    }
    S.cn = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) S.cn += __builtin_fabs(S.c[k]);
    S.status = ok ? kAlive : kInvalid;
    bool bad = false;
    int cur = 2 * D;  // the box faces hold at the starting corner
    if (lp >= 0 && ok) {
        // level D: the caller's rows against x, each checked to be finite
        while (cur < S.mt) {
            const int j = cur + S.gl;
            bool viol = false;
            if (j < S.mt) {
                const Row<D> r = S.row(j);
                bool fin = __builtin_isfinite(r.b);
#pragma unroll
                for (int k = 0; k < D; ++k) fin = fin && __builtin_isfinite(r.a[k]);
                bad |= !fin;
                viol = fin && Group<D, LG>::violates(r, S.x);
            }
            const uint64_t bal = __ballot(viol) & S.gmask;
            if (bal == 0) {
                cur += G;
                continue;
            }
            const int hv = cur + (__builtin_ctzll(bal) - S.gbase);
            S.template descend<D>(hv);
            if (S.status != kAlive) break;
            cur = hv + 1;
        }
        // an LP that died early still has its remaining rows checked for
        // non-finite values (INVALID takes precedence)
        if (S.status != kAlive)
            for (int j = cur + S.gl; j < S.mt; j += G) {
                const int64_t g = S.start + (j - 2 * D);
                bool fin = __builtin_isfinite(P.b[g]);
#pragma unroll
                for (int k = 0; k < D; ++k) fin = fin && __builtin_isfinite(P.a[k * P.num_constraints + g]);
                bad |= !fin;
            }
    }
    bad = (__ballot(bad) & S.gmask) != 0;
    if (lp >= 0 && S.gl == 0) {
        int status = bad ? kInvalid : S.status;
        double top = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) top = __builtin_fmax(top, __builtin_fabs(S.x[k]));
        if (status == kAlive) status = top >= P.M * (1.0 - 1e-9) ? kUnbounded : kOptimal;
        const bool has_x = status == kOptimal || status == kUnbounded;
#pragma unroll
        for (int k = 0; k < D; ++k) P.x_out[k * P.num_lps + lp] = has_x ? (float)S.x[k] : __builtin_nanf("");
        P.status[lp] = status;
    }
}

// Waves per SIMD the register allocation aims for: three for n = 4 (at most
// 168 VGPRs, a few spilled on the rare paths) hide more of the dependent FP64
// chains than two at ~180-220; for n = 5 the spills cost more than the third
// wave gains, so it keeps all the registers it needs.
template <int D>
constexpr int kWavesPerEu = D == 4 ? 3 : 1;

template <int D, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<D>))) void k_seidelN(ProblemN P) {
    constexpr int LG = G == 4 ? 2 : G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
    const int64_t q = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    solve_group<D, LG>(P, q < P.num_lps ? q : -1);
}

template <int D>
hipError_t launch(const ProblemN& P, int G, int64_t blocks, hipStream_t st) {
    switch (G) {
        case 4: hipLaunchKernelGGL((k_seidelN<D, 4>), dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        case 8: hipLaunchKernelGGL((k_seidelN<D, 8>), dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        case 16: hipLaunchKernelGGL((k_seidelN<D, 16>), dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        case 32: hipLaunchKernelGGL((k_seidelN<D, 32>), dim3((unsigned)blocks), dim3(256), 0, st, P); break;
        default: hipLaunchKernelGGL((k_seidelN<D, 64>), dim3((unsigned)blocks), dim3(256), 0, st, P); break;
    }
    return hipGetLastError();
}

}  // namespace rgbn

extern "C" rgb_err_t rgb_solven_batch(rgb_ctx_t* ctx, int32_t dim, int64_t num_lps, int64_t num_constraints,
                                      const int64_t* offsets, const float* a, const float* b, const float* c,
                                      double box, float* x_out, int32_t* status_out, int32_t lanes_per_lp,
                                      void* stream, void* ev_begin, void* ev_end) {
    if (!ctx || num_lps < 0 || num_constraints < 0) return RGB_ERR_INVALID_ARG;
    if (dim < 2 || dim > rgbn::kMaxDim) return RGB_ERR_INVALID_ARG;
    // the box must be positive and an FP32 value: x is written in FP32, and an
    // optimum on a face of a larger box would not be
    if (!(box > 0.0) || !(box <= 3.4028234663852886e38)) return RGB_ERR_INVALID_ARG;
    const int G = lanes_per_lp != 0 ? lanes_per_lp : dim == 5 ? 8 : 16;
    if (G != 4 && G != 8 && G != 16 && G != 32 && G != 64) return RGB_ERR_INVALID_ARG;
    if (num_lps > (int64_t(1) << 31) - 1) return RGB_ERR_TOO_LARGE;
    if (num_lps == 0) return RGB_OK;
    if (!offsets || !c || !x_out || !status_out) return RGB_ERR_INVALID_ARG;
    if (num_constraints > 0 && (!a || !b)) return RGB_ERR_INVALID_ARG;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return RGB_ERR_DEVICE;
    const int dev = rgb::ctx_device(ctx);
    if (dev != prev && hipSetDevice(dev) != hipSuccess) return RGB_ERR_DEVICE;
    rgbn::ProblemN P{offsets, a, b, c, x_out, status_out, num_lps, num_constraints, box};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t blocks = (num_lps * G + 255) / 256;
    if (ev_begin) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(ev_begin), st);
    hipError_t e = hipSuccess;
    switch (dim) {
        case 2: e = rgbn::launch<2>(P, G, blocks, st); break;
        case 3: e = rgbn::launch<3>(P, G, blocks, st); break;
        case 4: e = rgbn::launch<4>(P, G, blocks, st); break;
        default: e = rgbn::launch<5>(P, G, blocks, st); break;
    }
    if (ev_end) (void)hipEventRecord(reinterpret_cast<hipEvent_t>(ev_end), st);
    if (dev != prev) (void)hipSetDevice(prev);
    return e == hipSuccess ? RGB_OK : RGB_ERR_DEVICE;
}
