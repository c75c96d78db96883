/* TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for batched LPs in n
 * dimensions (n = 1..6).
 *
 * Only tests/ and the benchmark's CPU legs may call this code.  It shares
 * nothing with the HIP solver.
 *
 * Problem (Eq. (1)-(2) of the paper in n dimensions; the paper names higher
 * dimensions as its next step in Sec. 6):
 *
 *     maximize c.x over x in R^n subject to a_i.x <= b_i (i < m)
 *     and the bounding rows |x_k| <= M of Sec. 2.1 (M given, k = 1..n).
 *
 * The result is the lexicographically smallest maximiser: among the points
 * that maximise c.x, the one with the smallest x_1, then x_2, and so on.  The
 * box makes the feasible set compact, so it exists whenever the set is
 * non-empty.
 *
 * This file writes the definition out.  The feasible set is a polytope whose
 * vertices are intersections of n of its bounding hyperplanes (input rows and
 * box faces) with independent normals, and a linear objective (and the
 * lexicographic tie-break after it) is maximised at a vertex.  So: every
 * n-subset of hyperplanes, its intersection point by Gaussian elimination
 * with partial pivoting, kept if it satisfies every row, the best by
 * (c.v, -v_1, ..., -v_n).  O(m^(n+1)) per LP, FP64 throughout, with a
 * relative tolerance of 1e-10 on the feasibility test and 1e-12 on the
 * comparisons (the vertex is rounded).  A subset whose normals' determinant
 * is below 1e-14 times the product of their 1-norms has no single point.
 *
 * Status: INVALID when an input is not finite, n is out of range, M is not
 * finite and positive or the offsets are out of range; INFEASIBLE when no
 * vertex is feasible (or a row 0.x <= b has b < 0); UNBOUNDED when the optimum
 * lies on a face of the box (max_k |x_k| >= M (1 - 1e-9)): the LP without the
 * box is unbounded or has its optimum outside the box; OPTIMAL otherwise.  x
 * is reported for OPTIMAL and UNBOUNDED, NaN otherwise.  def names the n
 * hyperplanes of the optimal vertex: input rows 0..m-1, box faces -(2k+1)
 * (x_k <= M) and -(2k+2) (-x_k <= M) for k = 0..n-1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { OPTIMAL = 0, INFEASIBLE = 1, UNBOUNDED = 2, INVALID = 3 };
#define MAXD 6

typedef struct {
    double a[MAXD];
    double b;
    double na; /* |a|_1 */
    int id;
} plane;

/* Solve A v = r (n x n, A given by n planes) by Gaussian elimination with
 * partial pivoting.  Returns 0 when the determinant is below the singularity
 * threshold. */
static int intersect(int n, const plane *const *H, double *v) {
    double A[MAXD][MAXD + 1];
    double normprod = 1.0;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < n; ++k) A[i][k] = H[i]->a[k];
        A[i][n] = H[i]->b;
        normprod *= H[i]->na;
    }
    double det = 1.0;
    for (int col = 0; col < n; ++col) {
        int p = col;
        for (int i = col + 1; i < n; ++i)
            if (fabs(A[i][col]) > fabs(A[p][col])) p = i;
        if (A[p][col] == 0.0) return 0;
        if (p != col) {
            for (int k = 0; k <= n; ++k) {
                double t = A[p][k];
                A[p][k] = A[col][k];
                A[col][k] = t;
            }
            det = -det;
        }
        det *= A[col][col];
        for (int i = col + 1; i < n; ++i) {
            double f = A[i][col] / A[col][col];
            for (int k = col; k <= n; ++k) A[i][k] -= f * A[col][k];
        }
    }
    if (fabs(det) <= 1e-14 * normprod) return 0;
    for (int i = n - 1; i >= 0; --i) {
        double s = A[i][n];
        for (int k = i + 1; k < n; ++k) s -= A[i][k] * v[k];
        v[i] = s / A[i][i];
    }
    return 1;
}

/* does key (f, -v) beat (bf, -bv)?  Larger c.v first, then smaller x_1, x_2, ... */
static int better(int n, double f, const double *v, double bf, const double *bv, double scale) {
    double tol = 1e-12 * scale;
    if (f > bf + tol) return 1;
    if (f < bf - tol) return 0;
    for (int k = 0; k < n; ++k) {
        if (v[k] < bv[k] - tol) return 1;
        if (v[k] > bv[k] + tol) return 0;
    }
    return 0;
}

static void solve_one(int n, int64_t m, int64_t stride, const float *a, const float *b, const double *c, double M,
                      double *x, int32_t *status, int32_t *def) {
    for (int k = 0; k < n; ++k) {
        x[k] = NAN;
        def[k] = -100;
    }
    for (int k = 0; k < n; ++k)
        if (!isfinite(c[k])) {
            *status = INVALID;
            return;
        }
    for (int64_t i = 0; i < m; ++i) {
        int fin = isfinite(b[i]);
        for (int k = 0; k < n; ++k) fin &= isfinite(a[k * stride + i]) != 0;
        if (!fin) {
            *status = INVALID;
            return;
        }
    }
    plane *P = (plane *)malloc(sizeof(plane) * (size_t)(m + 2 * n));
    int np = 0;
    for (int64_t i = 0; i < m; ++i) {
        int zero = 1;
        double na = 0.0;
        for (int k = 0; k < n; ++k) {
            P[np].a[k] = a[k * stride + i];
            zero &= P[np].a[k] == 0.0;
            na += fabs(P[np].a[k]);
        }
        if (zero) {
            if (b[i] < 0.0) { /* 0 <= b fails: no point satisfies the row */
                free(P);
                *status = INFEASIBLE;
                return;
            }
            continue; /* 0 <= b holds everywhere */
        }
        P[np].b = b[i];
        P[np].na = na;
        P[np].id = (int)i;
        ++np;
    }
    for (int k = 0; k < n; ++k)
        for (int s = 0; s < 2; ++s) {
            for (int j = 0; j < n; ++j) P[np].a[j] = 0.0;
            P[np].a[k] = s == 0 ? 1.0 : -1.0;
            P[np].b = M;
            P[np].na = 1.0;
            P[np].id = -(2 * k + s + 1);
            ++np;
        }
    double cn = 0.0;
    for (int k = 0; k < n; ++k) cn += fabs(c[k]);
    int found = 0;
    double bf = 0.0, bv[MAXD] = {0.0};
    int bid[MAXD] = {0};
    int idx[MAXD];
    for (int k = 0; k < n; ++k) idx[k] = k;
    while (1) {
        const plane *H[MAXD];
        for (int k = 0; k < n; ++k) H[k] = &P[idx[k]];
        double v[MAXD];
        if (intersect(n, H, v)) {
            double vn = 0.0, f = 0.0;
            for (int k = 0; k < n; ++k) {
                vn += fabs(v[k]);
                f += c[k] * v[k];
            }
            double scale = cn * vn + vn + 1.0;
            /* the cheap key test first: a vertex that does not beat the best
               so far is never taken, feasible or not */
            if (!found || better(n, f, v, bf, bv, scale)) {
                int ok = 1;
                for (int j = 0; j < np && ok; ++j) {
                    double lhs = 0.0;
                    for (int k = 0; k < n; ++k) lhs += P[j].a[k] * v[k];
                    if (lhs - P[j].b > 1e-10 * (P[j].na * vn + fabs(P[j].b))) ok = 0;
                }
                if (ok) {
                    found = 1;
                    bf = f;
                    for (int k = 0; k < n; ++k) {
                        bv[k] = v[k];
                        bid[k] = H[k]->id;
                    }
                }
            }
        }
        /* next n-subset in lexicographic order */
        int k = n - 1;
        while (k >= 0 && idx[k] == np - n + k) --k;
        if (k < 0) break;
        ++idx[k];
        for (int j = k + 1; j < n; ++j) idx[j] = idx[j - 1] + 1;
    }
    free(P);
    if (!found) {
        *status = INFEASIBLE;
        return;
    }
    double top = 0.0;
    for (int k = 0; k < n; ++k) {
        x[k] = bv[k];
        def[k] = bid[k];
        top = fmax(top, fabs(bv[k]));
    }
    *status = top >= M * (1.0 - 1e-9) ? UNBOUNDED : OPTIMAL;
}

/* LPs [lp_begin, lp_end) of a CSR batch in n dimensions.  a is coordinate-
 * major (a[k * num_constraints + i] is component k of row i), c likewise
 * (c[k * num_lps + lp]); x and def are (B, n) row-major.  Returns -1 for n
 * out of range (nothing written), else 0. */
int rgb_oraclen_solve_range(int n, int64_t lp_begin, int64_t lp_end, int64_t num_lps, int64_t num_constraints,
                            const int64_t *offsets, const float *a, const float *b, const float *c, double M,
                            double *x, int32_t *status, int32_t *def) {
    if (n < 1 || n > MAXD) return -1;
    for (int64_t lp = lp_begin; lp < lp_end; ++lp) {
        int64_t s = offsets[lp], e = offsets[lp + 1];
        double cc[MAXD];
        for (int k = 0; k < n; ++k) cc[k] = c[k * num_lps + lp];
        if (!(isfinite(M) && M > 0.0) || s < 0 || e < s || e > num_constraints) {
            for (int k = 0; k < n; ++k) {
                x[n * lp + k] = NAN;
                def[n * lp + k] = -100;
            }
            status[lp] = INVALID;
            continue;
        }
        solve_one(n, e - s, num_constraints, a + s, b + s, cc, M, x + n * lp, status + lp, def + n * lp);
    }
    return 0;
}
