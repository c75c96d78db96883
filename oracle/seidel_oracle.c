/*
 * TEST INFRASTRUCTURE ONLY.  Plain, serial, FP64 reference for batched
 * two-dimensional linear programs, used to check the HIP solver.  Nothing in
 * the product path may link or call this file.
 *
 * Problem (Eq. (1)-(2), Sec. 2.1): maximize c.x subject to a_i.x <= b_i,
 * x in R^2.  Inputs are FP32 and are promoted exactly to FP64.
 *
 * Result definition.  x* is the lexicographically smallest maximiser of c.x
 * over P = {x : a_i.x <= b_i for all i}: among the maximisers take the
 * smallest x_1, then the smallest x_2.  The paper asks for a unique optimum
 * at every incremental step (Sec. 2.1) without naming the tie rule; the
 * lexicographic rule is the standard one.  status = INFEASIBLE if P is empty,
 * UNBOUNDED if P is non-empty and has no lexicographic optimum, OPTIMAL
 * otherwise.
 *
 * Method: Seidel's randomized incremental algorithm in the form of Sec. 2.1.
 *   - The bounding rows x <= M, x >= -M of Sec. 2.1 are kept symbolic
 *     (M -> infinity).  A state is either a POINT (the vertex of two input
 *     lines) or a RAY p + M*q.  The start is the box corner
 *     M*(s_x, s_y), s_j = +1 if c_j > 0 else -1.
 *   - Constraints are taken in input order (the random order Sec. 2.1 asks
 *     for is drawn by the input generator).  If the current state satisfies
 *     constraint i nothing changes; otherwise the new optimum lies on line i
 *     and is found by a 1D LP over the earlier constraints h < i (Eq. (3)
 *     u_left = max over left bounds, Eq. (4) u_right = min over right bounds).
 *   - Parallel earlier constraints either leave line i whole or empty it
 *     (Sec. 2.1); the 1D LP is infeasible if u_left > u_right (a single point
 *     is feasible).  The endpoint is picked by the objective, with the
 *     lexicographic rule when c is orthogonal to the line.
 *
 * Arithmetic.  Line l has direction u = (-a_l.y, a_l.x).  For h < l,
 * D_h = a_h.u = det(a_l, a_h) says whether h bounds line l from the right
 * (D_h > 0) or the left (D_h < 0), and the bound's position along u,
 * scaled by |a_l|^2, is N_h / D_h with
 *     N_h = b_h |a_l|^2 - b_l (a_l.a_h).
 * Bounds are compared by cross-multiplication and a vertex is kept as
 * homogeneous (X, Y, W) from Cramer's rule, so no decision divides.  Products
 * of two FP32 values are exact in FP64, hence D_h, det and c.u have exact
 * signs; for small integer inputs every decision here is exact.
 *
 * Range.  The solver under test computes in FP32, and the paper leaves the
 * precision open.  Reading taken: an LP whose incremental path visits a
 * vertex with a coordinate that rounds to an infinite FP32 value is INVALID
 * (outside the FP32 range), whatever the vertices that follow.
 *
 * Besides x* and status the oracle reports the defining pair, the number of
 * 1D LPs solved, and a margin: the smallest relative gap over the decisions it
 * took (violation tests of a vertex or of a ray along a parallel row,
 * parallel rows in a 1D LP, u_left vs u_right), +inf when no such decision
 * was taken.  Each gap is |lhs - rhs| over the sum of the magnitudes of the
 * terms both sides add up (for a vertex test |a_x X| + |a_y Y| + |b W|), the
 * scale of their rounding.  A margin near FP32 epsilon flags an LP whose
 * path FP32 arithmetic may not reproduce.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ST_OPTIMAL 0
#define ST_INFEASIBLE 1
#define ST_UNBOUNDED 2
#define ST_INVALID 3

#define K_CORNER 0 /* RAY from the origin towards the box corner (sx, sy) */
#define K_RAY 1    /* RAY along line l in direction dir * u_l */
#define K_POINT 2  /* vertex of lines l and h */

/* Gap of a decision lhs > rhs (or <) relative to the magnitudes of the terms
   the two sides are sums of: the rounding noise of a sum scales with them,
   not with the sum, which may cancel. */
static double relgap(double lhs, double rhs, double scale) {
    if (scale == 0.0) return 0.0;
    return fabs(lhs - rhs) / scale;
}

static void lower_margin(double *margin, double g) {
    if (g < *margin) *margin = g;
}

typedef struct {
    double x, y;
    int32_t status, def_i, def_j, def_k, n_1dlp;
    double margin;
} lp_result;

static lp_result solve_one(int64_t m, const float *ax, const float *ay, const float *b, float cxf,
                           float cyf) {
    lp_result res;
    res.x = NAN;
    res.y = NAN;
    res.status = ST_OPTIMAL;
    res.def_i = -1;
    res.def_j = -1;
    res.def_k = -1;
    res.n_1dlp = 0;
    res.margin = INFINITY;

    double cx = cxf, cy = cyf;
    if (!isfinite(cx) || !isfinite(cy)) {
        res.status = ST_INVALID;
        return res;
    }
    for (int64_t i = 0; i < m; ++i) {
        if (!isfinite(ax[i]) || !isfinite(ay[i]) || !isfinite(b[i])) {
            res.status = ST_INVALID;
            return res;
        }
    }

    int kind = K_CORNER;
    double sx = cx > 0.0 ? 1.0 : -1.0;
    double sy = cy > 0.0 ? 1.0 : -1.0;
    int64_t l = -1, h = -1;
    double dir = 0.0;
    double X = 0.0, Y = 0.0, W = 1.0; /* vertex = (X/W, Y/W), W > 0 */

    for (int64_t i = 0; i < m; ++i) {
        double aix = ax[i], aiy = ay[i], bi = b[i];

        if (aix == 0.0 && aiy == 0.0) {
            /* 0 <= b_i: holds everywhere or nowhere (an exact decision) */
            if (bi < 0.0) {
                res.status = ST_INFEASIBLE;
                res.def_i = (int32_t)i;
                return res;
            }
            continue;
        }

        int violated;
        if (kind == K_CORNER) {
            double t = sx * aix + sy * aiy;
            violated = t > 0.0 || (t == 0.0 && 0.0 > bi); /* exact in FP64 */
        } else if (kind == K_RAY) {
            double alx = ax[l], aly = ay[l], bl = b[l];
            double t = dir * (alx * aiy - aly * aix); /* a_i . (dir * u_l) */
            if (t != 0.0) {
                violated = t > 0.0;
            } else {
                /* a_i parallel to a_l: compare a_i.p0 with b_i, p0 = b_l a_l / |a_l|^2 */
                double lhs = bl * (aix * alx + aiy * aly);
                double rhs = bi * (alx * alx + aly * aly);
                violated = lhs > rhs;
                lower_margin(&res.margin,
                             relgap(lhs, rhs, fabs(bl) * (fabs(aix * alx) + fabs(aiy * aly)) + fabs(rhs)));
            }
        } else {
            double lhs = aix * X + aiy * Y;
            double rhs = bi * W;
            violated = lhs > rhs;
            lower_margin(&res.margin, relgap(lhs, rhs, fabs(aix * X) + fabs(aiy * Y) + fabs(rhs)));
        }
        if (!violated) continue;

        /* 1D LP on line i over the constraints h < i (Eq. (3)-(4)) */
        res.n_1dlp++;
        double nrm2 = aix * aix + aiy * aiy;
        int64_t hi = -1, lo = -1;
        double hiN = 0.0, hiD = 1.0, loN = 0.0, loD = -1.0;
        double hiS = 0.0, loS = 0.0; /* magnitudes of the terms of hiN, loN */
        for (int64_t j = 0; j < i; ++j) {
            double ajx = ax[j], ajy = ay[j], bj = b[j];
            double D = aix * ajy - aiy * ajx;
            double dotp = aix * ajx + aiy * ajy;
            double N = bj * nrm2 - bi * dotp;
            double S = fabs(bj * nrm2) + fabs(bi) * (fabs(aix * ajx) + fabs(aiy * ajy));
            if (D > 0.0) {
                if (hi < 0 || N * hiD < hiN * D) { hi = j; hiN = N; hiD = D; hiS = S; }
            } else if (D < 0.0) {
                if (lo < 0 || N * loD > loN * D) { lo = j; loN = N; loD = D; loS = S; }
            } else {
                /* parallel (or zero normal): line i lies inside h iff N >= 0 */
                if (ajx != 0.0 || ajy != 0.0) lower_margin(&res.margin, relgap(bj * nrm2, bi * dotp, S));
                if (N < 0.0) {
                    res.status = ST_INFEASIBLE;
                    res.def_i = (int32_t)i;
                    res.def_j = (int32_t)j;
                    return res;
                }
            }
        }
        if (hi >= 0 && lo >= 0) {
            /* u_left > u_right  <=>  loN/loD > hiN/hiD  <=>  loN*hiD < hiN*loD (loD < 0 < hiD) */
            double lhs = loN * hiD, rhs = hiN * loD;
            lower_margin(&res.margin, relgap(lhs, rhs, loS * hiD - hiS * loD));
            if (lhs < rhs) {
                res.status = ST_INFEASIBLE;
                res.def_i = (int32_t)i;
                res.def_j = (int32_t)lo;
                res.def_k = (int32_t)hi;
                return res;
            }
        }
        /* direction of improvement along u = (-a_i.y, a_i.x): first non-zero of
           (c.u, -u.x, -u.y); -u.x = a_i.y, -u.y = -a_i.x */
        double cu = cy * aix - cx * aiy;
        double s;
        if (cu != 0.0) s = cu > 0.0 ? 1.0 : -1.0;
        else if (aiy != 0.0) s = aiy > 0.0 ? 1.0 : -1.0;
        else s = -aix > 0.0 ? 1.0 : -1.0;

        int64_t pick = s > 0.0 ? hi : lo;
        l = i;
        if (pick < 0) {
            kind = K_RAY;
            dir = s;
        } else {
            kind = K_POINT;
            h = pick;
            double ahx = ax[h], ahy = ay[h], bh = b[h];
            X = bi * ahy - bh * aiy;
            Y = aix * bh - ahx * bi;
            W = aix * ahy - aiy * ahx;
            if (W < 0.0) { X = -X; Y = -Y; W = -W; }
            /* a vertex whose coordinates round to an infinite FP32 value lies
               outside what an FP32 solver can represent: the LP is INVALID */
            if (isinf((float)(X / W)) || isinf((float)(Y / W))) {
                res.status = ST_INVALID;
                res.def_i = (int32_t)i;
                res.def_j = (int32_t)h;
                return res;
            }
        }
    }

    if (kind == K_POINT) {
        res.status = ST_OPTIMAL;
        res.x = X / W;
        res.y = Y / W;
        res.def_i = (int32_t)l;
        res.def_j = (int32_t)h;
    } else {
        res.status = ST_UNBOUNDED;
        res.def_i = (int32_t)l;
        res.def_j = kind == K_RAY ? (int32_t)dir : 0;
    }
    return res;
}

/*
 * Solve LPs [lp_begin, lp_end) of a CSR-offset SoA batch.  offsets must be
 * non-decreasing with offsets[0] = 0; all arrays are host memory owned by the
 * caller.  The optional outputs (def_i, def_j, def_k, n_1dlp, margin) may be
 * NULL.  def_*: OPTIMAL -> the two lines through x*; INFEASIBLE -> the line
 * whose 1D LP failed and the one or two earlier lines that empty it (a
 * certificate of at most three constraints); UNBOUNDED -> def_i is the
 * ray's line and def_j its direction (+1 or -1 times u_l), or -1 and 0 for
 * the initial box-corner ray.
 * Returns 0, or -1 if offsets are malformed for an LP in range (that LP gets
 * status INVALID).
 */
int rgb_oracle_solve_range(int64_t lp_begin, int64_t lp_end, const int64_t *offsets, const float *ax,
                           const float *ay, const float *b, const float *cx, const float *cy,
                           double *x_out, double *y_out, int32_t *status, int32_t *def_i,
                           int32_t *def_j, int32_t *def_k, int32_t *n_1dlp, double *margin) {
    int rc = 0;
    for (int64_t k = lp_begin; k < lp_end; ++k) {
        int64_t s = offsets[k], e = offsets[k + 1];
        lp_result r;
        if (s < 0 || e < s) {
            memset(&r, 0, sizeof(r));
            r.x = NAN;
            r.y = NAN;
            r.status = ST_INVALID;
            r.def_i = r.def_j = r.def_k = -1;
            r.margin = INFINITY;
            rc = -1;
        } else {
            r = solve_one(e - s, ax + s, ay + s, b + s, cx[k], cy[k]);
        }
        x_out[k] = r.x;
        y_out[k] = r.y;
        status[k] = r.status;
        if (def_i) def_i[k] = r.def_i;
        if (def_j) def_j[k] = r.def_j;
        if (def_k) def_k[k] = r.def_k;
        if (n_1dlp) n_1dlp[k] = r.n_1dlp;
        if (margin) margin[k] = r.margin;
    }
    return rc;
}
