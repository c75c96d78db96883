"""Test helpers: golden-file parsing, result comparison and independent
certificate checks in exact rational arithmetic."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

OPTIMAL, INFEASIBLE, UNBOUNDED, INVALID = 0, 1, 2, 3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Parity bar: status bit-exact; for OPTIMAL LPs ||x - x_ref|| <= 1e-4 * max(1, ||x_ref||).
X_RTOL = 1e-4


def parse_golden(path):
    lps, cur = [], None
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "lp":
                cur = {"name": tok[1], "rows": [], "c": None, "expect": None}
            elif tok[0] == "c":
                cur["c"] = (float(tok[1]), float(tok[2]))
            elif tok[0] == "row":
                cur["rows"].append(tuple(float(t) for t in tok[1:4]))
            elif tok[0] == "expect":
                st = {"optimal": OPTIMAL, "infeasible": INFEASIBLE, "unbounded": UNBOUNDED}[tok[1]]
                xy = (float(tok[2]), float(tok[3])) if st == OPTIMAL else None
                cur["expect"] = (st, xy)
            elif tok[0] == "end":
                lps.append(cur)
                cur = None
    return lps


def golden_batch(path):
    """Turn a golden file into a gen.Batch plus the expected (status, xy) list."""
    from paper_1902_04995_amd import gen
    lps = parse_golden(path)
    sizes = [len(lp["rows"]) for lp in lps]
    offs = np.zeros(len(lps) + 1, np.int64)
    np.cumsum(sizes, out=offs[1:])
    rows = np.array([r for lp in lps for r in lp["rows"]], np.float64).reshape(-1, 3)
    bt = gen.Batch(offs, rows[:, 0].astype(np.float32), rows[:, 1].astype(np.float32),
                   rows[:, 2].astype(np.float32),
                   np.array([lp["c"][0] for lp in lps], np.float32),
                   np.array([lp["c"][1] for lp in lps], np.float32),
                   np.full(len(lps), gen.KIND_OTHER, np.int8), os.path.basename(path))
    return bt, [lp["expect"] for lp in lps], [lp["name"] for lp in lps]


def rows_batch(lps, name="rows"):
    """A gen.Batch from a list of (rows, (cx, cy)) with rows = [(ax, ay, b), ...]
    given as Python or numpy floats (rounded to FP32)."""
    from paper_1902_04995_amd import gen
    sizes = [len(r) for r, _ in lps]
    offs = np.zeros(len(lps) + 1, np.int64)
    np.cumsum(sizes, out=offs[1:])
    flat = np.array([x for r, _ in lps for x in r], np.float64).reshape(-1, 3)
    return gen.Batch(offs, flat[:, 0].astype(np.float32), flat[:, 1].astype(np.float32),
                     flat[:, 2].astype(np.float32), np.array([c[0] for _, c in lps], np.float32),
                     np.array([c[1] for _, c in lps], np.float32), np.full(len(lps), gen.KIND_OTHER, np.int8), name)


# LPs whose smallest decision gap in the oracle is below this may take another
# path in FP32 (a different count of 1D LPs); their count is not compared.
N1D_MARGIN = 1e-5


def compare_n1d(n1d, ref, margin=N1D_MARGIN):
    """(indices where the GPU's count of 1D LPs differs from the oracle's,
    number of LPs left out) over LPs that are not INVALID and whose oracle
    margin is at least `margin`."""
    n1d = np.asarray(n1d)
    keep = (np.asarray(ref["status"]) != INVALID) & (np.asarray(ref["margin"]) >= margin)
    bad = np.flatnonzero(keep & (n1d != np.asarray(ref["n_1dlp"])))
    return bad, int((~keep & (np.asarray(ref["status"]) != INVALID)).sum())


def compare(status, x, y, ref_status, ref_x, ref_y, rtol=X_RTOL):
    """Indices where (status, x) disagrees with the reference under the parity bar."""
    status = np.asarray(status)
    ref_status = np.asarray(ref_status)
    bad_status = status != ref_status
    opt = (ref_status == OPTIMAL) & ~bad_status
    dx = np.hypot(np.asarray(x, np.float64) - ref_x, np.asarray(y, np.float64) - ref_y)
    scale = np.maximum(1.0, np.hypot(ref_x, ref_y))
    bad_x = np.zeros_like(bad_status)
    bad_x[opt] = ~(dx[opt] <= rtol * scale[opt])
    return np.flatnonzero(bad_status), np.flatnonzero(bad_x)


def F(v):
    return Fraction(float(v))


def exact_infeasible(rows):
    """Exact emptiness test of {x: a.x <= b for (a, b) in rows} for <= 3 rows
    (Helly in the plane: a certificate needs at most three)."""
    import oracle
    ax = [r[0] for r in rows]
    ay = [r[1] for r in rows]
    b = [r[2] for r in rows]
    st, _, _ = oracle.brute_force(ax, ay, b, 0.0, 0.0)
    return st == INFEASIBLE


def check_optimal_certificate(ax, ay, b, cx, cy, x, y, i, j, feas_tol=1e-9):
    """x* feasible (max violation <= feas_tol * scale), lines i and j tight at
    x*, and c in the cone of a_i, a_j (c = l_i a_i + l_j a_j, l >= 0).
    Returns an error string or None."""
    ax = np.asarray(ax, np.float64)
    ay = np.asarray(ay, np.float64)
    b = np.asarray(b, np.float64)
    viol = ax * x + ay * y - b
    scale = np.abs(ax * x) + np.abs(ay * y) + np.abs(b) + 1e-300
    if np.any(viol > feas_tol * scale):
        return f"infeasible x*: max rel violation {np.max(viol / scale):.3e}"
    for k in (i, j):
        if abs(viol[k]) > feas_tol * scale[k]:
            return f"defining line {k} not tight ({viol[k]:.3e})"
    det = ax[i] * ay[j] - ay[i] * ax[j]
    if det == 0:
        return "parallel defining pair"
    li = (cx * ay[j] - cy * ax[j]) / det
    lj = (ax[i] * cy - ay[i] * cx) / det
    tol = 1e-12 * (abs(cx) + abs(cy) + 1.0)
    if li < -tol or lj < -tol:
        return f"c outside the normal cone (l = {li:.3e}, {lj:.3e})"
    return None


def check_unbounded_ray(ax, ay, b, cx, cy, l, dirn):
    """Exact check of an unbounded certificate: the ray p0 + t d lies in P for
    all large t (so P is non-empty and recedes along d) and
    (c.d, -d1, -d2) >_lex 0.  Line l gives p0 = b_l a_l / |a_l|^2 and
    d = dirn * (-a_l.y, a_l.x); l < 0 stands for the box-corner start
    p0 = 0, d = (s_x, s_y)."""
    if l < 0:
        p0 = (Fraction(0), Fraction(0))
        d = (Fraction(1 if cx > 0 else -1), Fraction(1 if cy > 0 else -1))
    else:
        alx, aly, bl = F(ax[l]), F(ay[l]), F(b[l])
        n2 = alx * alx + aly * aly
        p0 = (bl * alx / n2, bl * aly / n2)
        d = (-aly * dirn, alx * dirn)
    for p, q, r in zip(ax, ay, b):
        p, q, r = F(p), F(q), F(r)
        ad = p * d[0] + q * d[1]
        if ad > 0 or (ad == 0 and p * p0[0] + q * p0[1] > r):
            return "the ray leaves P"
    key = (F(cx) * d[0] + F(cy) * d[1], -d[0], -d[1])
    if not key > (0, 0, 0):
        return "ray does not improve the objective"
    return None


def parse_golden3(path):
    """3D fixtures: lp NAME / c cx cy cz / box M / row ax ay az b ... /
    expect optimal|unbounded x y z  or  expect infeasible / end."""
    lps, cur = [], None
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "lp":
                cur = {"name": tok[1], "rows": [], "c": None, "box": None, "expect": None}
            elif tok[0] == "c":
                cur["c"] = tuple(float(t) for t in tok[1:4])
            elif tok[0] == "box":
                cur["box"] = float(tok[1])
            elif tok[0] == "row":
                cur["rows"].append(tuple(float(t) for t in tok[1:5]))
            elif tok[0] == "expect":
                st = {"optimal": OPTIMAL, "infeasible": INFEASIBLE, "unbounded": UNBOUNDED}[tok[1]]
                xyz = tuple(float(t) for t in tok[2:5]) if st != INFEASIBLE else None
                cur["expect"] = (st, xyz)
            elif tok[0] == "end":
                lps.append(cur)
                cur = None
    return lps


def golden3_batch(lps):
    """One Batch3 holding the fixtures (they must share one box)."""
    from paper_1902_04995_amd import gen3
    parts = []
    for lp in lps:
        rows = np.array(lp["rows"], dtype=np.float32).reshape(-1, 4)
        offs = np.array([0, rows.shape[0]], dtype=np.int64)
        c = np.array(lp["c"], dtype=np.float32)
        parts.append(gen3.Batch3(offs, rows[:, 0].copy(), rows[:, 1].copy(), rows[:, 2].copy(), rows[:, 3].copy(),
                                 c[:1], c[1:2], c[2:], np.zeros(1, np.int8), lp["box"], lp["name"]))
    return parts


def kkt_residual3(A, b, c, x, tight_tol=1e-7):
    """Optimality certificate for a 3D LP without the box: the rows tight at x
    (|a.x - b| <= tight_tol (1 + |b|)) must carry multipliers lambda >= 0 with
    sum lambda a = c.  Returns (max violation of a.x <= b, relative residual of
    the non-negative least-squares fit)."""
    from scipy.optimize import nnls
    slack = A @ x - b
    viol = float(np.max(slack, initial=-np.inf))
    tight = np.abs(slack) <= tight_tol * (1.0 + np.abs(b))
    if not tight.any():
        return viol, float(np.linalg.norm(c))
    lam, res = nnls(A[tight].T, c)
    return viol, float(res / max(1e-300, np.linalg.norm(c)))


def parse_golden_n(path):
    """n-dimensional fixtures: lp NAME / dim n / c c_1 .. c_n / box M /
    row a_1 .. a_n b ... / expect optimal|unbounded x_1 .. x_n  or
    expect infeasible / end."""
    lps, cur = [], None
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "lp":
                cur = {"name": tok[1], "rows": [], "c": None, "box": None, "expect": None, "dim": None}
            elif tok[0] == "dim":
                cur["dim"] = int(tok[1])
            elif tok[0] == "c":
                cur["c"] = tuple(float(t) for t in tok[1:])
            elif tok[0] == "box":
                cur["box"] = float(tok[1])
            elif tok[0] == "row":
                cur["rows"].append(tuple(float(t) for t in tok[1:]))
            elif tok[0] == "expect":
                st = {"optimal": OPTIMAL, "infeasible": INFEASIBLE, "unbounded": UNBOUNDED}[tok[1]]
                x = tuple(float(t) for t in tok[2:]) if st != INFEASIBLE else None
                cur["expect"] = (st, x)
            elif tok[0] == "end":
                n = cur["dim"]
                assert len(cur["c"]) == n and all(len(r) == n + 1 for r in cur["rows"]), cur["name"]
                assert cur["expect"][1] is None or len(cur["expect"][1]) == n, cur["name"]
                lps.append(cur)
                cur = None
    return lps


def golden_n_batch(lp):
    """A one-LP BatchN holding one fixture."""
    from paper_1902_04995_amd import genn
    n = lp["dim"]
    rows = np.array(lp["rows"], dtype=np.float64).reshape(-1, n + 1)
    return genn.from_rows([rows], [lp["c"]], lp["box"], name=lp["name"])
