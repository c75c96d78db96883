/* TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for batched 3D LPs.
 *
 * Only tests/ and the benchmark's CPU legs may call this code.  It shares
 * nothing with the HIP solver.
 *
 * Problem (Eq. (1)-(2) of the paper with n = 3; the paper names higher
 * dimensions as its next step in Sec. 6):
 *
 *     maximize c.x over x in R^3 subject to a_i.x <= b_i (i < m)
 *     and the bounding rows |x_k| <= M of Sec. 2.1 (M given, k = 1..3).
 *
 * The result is the lexicographically smallest maximiser: among the points
 * that maximise c.x, the one with the smallest x, then y, then z.  The box
 * makes the feasible set compact, so it exists whenever the set is non-empty.
 *
 * This file writes the definition out.  The feasible set is a polytope whose
 * vertices are intersections of three of its bounding planes (input rows and
 * box faces) with independent normals, and a linear objective (and the
 * lexicographic tie-break after it) is maximised at a vertex.  So: every
 * triple of planes, its intersection point by Cramer's rule, kept if it
 * satisfies every row, the best by (c.v, -v_x, -v_y, -v_z).  O(m^4) per LP,
 * FP64 throughout, with a relative tolerance of 1e-10 on the feasibility test
 * and 1e-12 on the comparisons (the vertex is rounded).
 *
 * Status: INVALID when an input is not finite, M is not finite and positive
 * or the offsets are out of range; INFEASIBLE when no vertex is feasible (or
 * a row 0.x <= b has b < 0); UNBOUNDED when the optimum lies on a face of the
 * box (max_k |x_k| >= M (1 - 1e-9)): the LP without the box is unbounded or
 * has its optimum outside the box; OPTIMAL otherwise.  x is reported for
 * OPTIMAL and UNBOUNDED, NaN otherwise.  def_* name the three planes of the
 * optimal vertex: input rows 0..m-1, box faces -1 (x <= M), -2 (-x <= M),
 * -3 (y <= M), -4 (-y <= M), -5 (z <= M), -6 (-z <= M).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { OPTIMAL = 0, INFEASIBLE = 1, UNBOUNDED = 2, INVALID = 3 };

typedef struct {
    double a[3];
    double b;
    double na;  /* |a|_1 */
    int id;
} plane;

static double det3(const double *p, const double *q, const double *r) {
    return p[0] * (q[1] * r[2] - q[2] * r[1]) - p[1] * (q[0] * r[2] - q[2] * r[0]) +
           p[2] * (q[0] * r[1] - q[1] * r[0]);
}

/* does key (f, -v) beat (bf, -bv)?  Larger c.v first, then smaller x, y, z */
static int better(double f, const double *v, double bf, const double *bv, double scale) {
    double tol = 1e-12 * scale;
    if (f > bf + tol) return 1;
    if (f < bf - tol) return 0;
    for (int k = 0; k < 3; ++k) {
        if (v[k] < bv[k] - tol) return 1;
        if (v[k] > bv[k] + tol) return 0;
    }
    return 0;
}

static void solve_one(int64_t m, const float *ax, const float *ay, const float *az, const float *b, const double *c,
                      double M, double *x, int32_t *status, int32_t *def) {
    x[0] = x[1] = x[2] = NAN;
    def[0] = def[1] = def[2] = -100;
    if (!isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2])) {
        *status = INVALID;
        return;
    }
    for (int64_t i = 0; i < m; ++i)
        if (!isfinite(ax[i]) || !isfinite(ay[i]) || !isfinite(az[i]) || !isfinite(b[i])) {
            *status = INVALID;
            return;
        }
    plane *P = (plane *)malloc(sizeof(plane) * (size_t)(m + 6));
    int n = 0;
    for (int64_t i = 0; i < m; ++i) {
        double a0 = ax[i], a1 = ay[i], a2 = az[i], bi = b[i];
        if (a0 == 0.0 && a1 == 0.0 && a2 == 0.0) {
            if (bi < 0.0) {  /* 0 <= b fails: no point satisfies the row */
                free(P);
                *status = INFEASIBLE;
                return;
            }
            continue;  /* 0 <= b holds everywhere */
        }
        P[n].a[0] = a0;
        P[n].a[1] = a1;
        P[n].a[2] = a2;
        P[n].b = bi;
        P[n].na = fabs(a0) + fabs(a1) + fabs(a2);
        P[n].id = (int)i;
        ++n;
    }
    for (int k = 0; k < 3; ++k)
        for (int s = 0; s < 2; ++s) {
            P[n].a[0] = P[n].a[1] = P[n].a[2] = 0.0;
            P[n].a[k] = s == 0 ? 1.0 : -1.0;
            P[n].b = M;
            P[n].na = 1.0;
            P[n].id = -(2 * k + s + 1);
            ++n;
        }
    double cn = fabs(c[0]) + fabs(c[1]) + fabs(c[2]);
    int found = 0;
    double bf = 0.0, bv[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q)
            for (int r = q + 1; r < n; ++r) {
                const double *A = P[p].a, *B = P[q].a, *C = P[r].a;
                double D = det3(A, B, C);
                if (fabs(D) <= 1e-14 * P[p].na * P[q].na * P[r].na) continue;  /* no single point */
                /* Cramer: replace one column of [A; B; C] by (b_p, b_q, b_r) */
                double rhs[3] = {P[p].b, P[q].b, P[r].b};
                double v[3];
                for (int k = 0; k < 3; ++k) {
                    double A2[3] = {A[0], A[1], A[2]}, B2[3] = {B[0], B[1], B[2]}, C2[3] = {C[0], C[1], C[2]};
                    A2[k] = rhs[0];
                    B2[k] = rhs[1];
                    C2[k] = rhs[2];
                    v[k] = det3(A2, B2, C2) / D;
                }
                double vn = fabs(v[0]) + fabs(v[1]) + fabs(v[2]);
                double f = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
                double scale = cn * vn + vn + 1.0;
                /* the cheap key test first: a vertex that does not beat the
                   best so far is never taken, feasible or not */
                if (found && !better(f, v, bf, bv, scale)) continue;
                int ok = 1;
                for (int j = 0; j < n && ok; ++j) {
                    double lhs = P[j].a[0] * v[0] + P[j].a[1] * v[1] + P[j].a[2] * v[2];
                    if (lhs - P[j].b > 1e-10 * (P[j].na * vn + fabs(P[j].b))) ok = 0;
                }
                if (ok) {
                    found = 1;
                    bf = f;
                    bv[0] = v[0];
                    bv[1] = v[1];
                    bv[2] = v[2];
                    def[0] = P[p].id;
                    def[1] = P[q].id;
                    def[2] = P[r].id;
                }
            }
    free(P);
    if (!found) {
        def[0] = def[1] = def[2] = -100;
        *status = INFEASIBLE;
        return;
    }
    x[0] = bv[0];
    x[1] = bv[1];
    x[2] = bv[2];
    double top = fmax(fabs(bv[0]), fmax(fabs(bv[1]), fabs(bv[2])));
    *status = top >= M * (1.0 - 1e-9) ? UNBOUNDED : OPTIMAL;
}

/* LPs [lp_begin, lp_end) of a CSR batch; x is (B, 3) row-major, def (B, 3). */
int rgb_oracle3_solve_range(int64_t lp_begin, int64_t lp_end, int64_t num_constraints, const int64_t *offsets,
                            const float *ax, const float *ay, const float *az, const float *b, const float *cx,
                            const float *cy, const float *cz, double M, double *x, int32_t *status, int32_t *def) {
    for (int64_t k = lp_begin; k < lp_end; ++k) {
        int64_t s = offsets[k], e = offsets[k + 1];
        double c[3] = {cx[k], cy[k], cz[k]};
        if (!(isfinite(M) && M > 0.0) || s < 0 || e < s || e > num_constraints) {
            x[3 * k] = x[3 * k + 1] = x[3 * k + 2] = NAN;
            def[3 * k] = def[3 * k + 1] = def[3 * k + 2] = -100;
            status[k] = INVALID;
            continue;
        }
        solve_one(e - s, ax + s, ay + s, az + s, b + s, c, M, x + 3 * k, status + k, def + 3 * k);
    }
    return 0;
}
