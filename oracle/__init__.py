"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for batched 2D LPs.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP solver.

Contents
  * ``solve``      - serial FP64 Seidel in C (``seidel_oracle.c``), driven over
                     LP ranges by Python threads (ctypes drops the GIL).
  * ``brute_force`` - exact rational vertex enumeration for one small LP; the
                     pin the oracle is checked against.
  * ``solve3``     - 3D LPs inside a box: FP64 vertex enumeration in C
                     (``lp3_oracle.c``), the definition written out.
  * ``brute_force3`` - the same definition in exact rational arithmetic for
                     one small LP.
  * ``solve_n``    - LPs in n dimensions (n = 1..6) inside a box: FP64 vertex
                     enumeration in C (``lpn_oracle.c``), the definition
                     written out for any n.
  * ``brute_force_n`` - that definition in exact rational arithmetic.
  * ``build``      - compiles the C files with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from fractions import Fraction

import numpy as np

OPTIMAL, INFEASIBLE, UNBOUNDED, INVALID = 0, 1, 2, 3
STATUS_NAMES = {OPTIMAL: "optimal", INFEASIBLE: "infeasible", UNBOUNDED: "unbounded", INVALID: "invalid"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "seidel_oracle.c")
_LIB = os.path.join(_HERE, "librgb_oracle.so")
_SRC3 = os.path.join(_HERE, "lp3_oracle.c")
_LIB3 = os.path.join(_HERE, "librgb_oracle3.so")
_SRCN = os.path.join(_HERE, "lpn_oracle.c")
_LIBN = os.path.join(_HERE, "librgb_oraclen.so")
_lib = None
_lib3 = None
_libn = None


def build(force: bool = True) -> str:
    """Compile the oracle.  -ffp-contract=off keeps every product and sum
    rounded as written (no fused multiply-add)."""
    for src, lib in ((_SRC, _LIB), (_SRC3, _LIB3), (_SRCN, _LIBN)):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                                   "-shared", "-o", tmp, src, "-lm"])
            os.replace(tmp, lib)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        f = lib.rgb_oracle_solve_range
        P = ctypes.c_void_p
        f.argtypes = [ctypes.c_int64, ctypes.c_int64] + [P] * 14
        f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def solve(batch, threads: int | None = None, lp_begin: int = 0, lp_end: int | None = None):
    """Solve LPs [lp_begin, lp_end) of ``batch`` (a ``gen.Batch`` or any object
    with offsets/ax/ay/b/cx/cy).  Returns a dict with x, y (float64), status,
    def_i, def_j, def_k, n_1dlp (int32) and margin (float64), indexed like
    the batch, plus the thread count used.  LPs are split over ``threads`` by
    equal total constraint count."""
    lib = _load()
    offsets = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    ax = np.ascontiguousarray(batch.ax, dtype=np.float32)
    ay = np.ascontiguousarray(batch.ay, dtype=np.float32)
    b = np.ascontiguousarray(batch.b, dtype=np.float32)
    cx = np.ascontiguousarray(batch.cx, dtype=np.float32)
    cy = np.ascontiguousarray(batch.cy, dtype=np.float32)
    B = offsets.shape[0] - 1
    if lp_end is None:
        lp_end = B
    out = {
        "x": np.full(B, np.nan), "y": np.full(B, np.nan),
        "status": np.full(B, INVALID, dtype=np.int32),
        "def_i": np.full(B, -1, dtype=np.int32), "def_j": np.full(B, -1, dtype=np.int32),
        "def_k": np.full(B, -1, dtype=np.int32),
        "n_1dlp": np.zeros(B, dtype=np.int32), "margin": np.full(B, np.inf),
    }
    if threads is None:
        threads = max(1, len(os.sched_getaffinity(0)))
    n = lp_end - lp_begin
    if n <= 0:
        return out
    threads = max(1, min(threads, n))
    # split by equal sum of m (the oracle's cost is ~linear in m on random order)
    work = offsets[lp_begin:lp_end + 1] - offsets[lp_begin]
    cuts = np.searchsorted(work, np.linspace(0, work[-1], threads + 1)[1:-1]) + lp_begin
    bounds = [lp_begin] + sorted(set(int(c) for c in cuts)) + [lp_end]
    args = [_ptr(a) for a in (offsets, ax, ay, b, cx, cy, out["x"], out["y"], out["status"],
                               out["def_i"], out["def_j"], out["def_k"], out["n_1dlp"], out["margin"])]

    def run(s, e):
        if e > s:
            lib.rgb_oracle_solve_range(s, e, *args)

    if len(bounds) == 2:
        run(bounds[0], bounds[1])
    else:
        ths = [threading.Thread(target=run, args=(bounds[i], bounds[i + 1])) for i in range(len(bounds) - 1)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    out["threads"] = len(bounds) - 1
    return out


# ---------------------------------------------------------------------------
# Exact brute force (the pin).  Same result definition as the C oracle:
# x* = lexicographically smallest maximiser of c.x over P.  Every vertex of
# P intersected with a box |x_j| <= R is a pairwise intersection of input
# lines and box lines; R is chosen beyond every such vertex and every line's
# distance from the origin.  With the perturbed objective
# c_eps = c - eps*e1 - eps^2*e2 (eps -> 0+) the optimum over the box-clipped
# P is the lexicographic maximum of (c.v, -v1, -v2) over its vertices; it
# touches the box iff the LP has no lexicographic optimum.
# ---------------------------------------------------------------------------

def _frac(v) -> Fraction:
    return Fraction(float(v))


def brute_force(ax, ay, b, cx, cy):
    """Returns (status, x, y) with x, y exact Fractions (None unless OPTIMAL)."""
    A = [(_frac(p), _frac(q), _frac(r)) for p, q, r in zip(ax, ay, b)]
    c = (_frac(cx), _frac(cy))
    for p, q, r in A:
        if p == 0 and q == 0 and r < 0:
            return INFEASIBLE, None, None
    lines = [(p, q, r) for p, q, r in A if not (p == 0 and q == 0)]
    # radius: beyond every vertex of the input lines and every line's nearest point
    big = Fraction(1)
    for i in range(len(lines)):
        p1, q1, r1 = lines[i]
        n1 = abs(p1) + abs(q1)
        big = max(big, abs(r1) / n1 * 2)
        for j in range(i + 1, len(lines)):
            p2, q2, r2 = lines[j]
            det = p1 * q2 - q1 * p2
            if det != 0:
                x = (r1 * q2 - r2 * q1) / det
                y = (p1 * r2 - p2 * r1) / det
                big = max(big, abs(x), abs(y))
    R = 4 * big + 4
    box = [(Fraction(1), Fraction(0), R), (Fraction(-1), Fraction(0), R),
           (Fraction(0), Fraction(1), R), (Fraction(0), Fraction(-1), R)]
    allL = lines + box

    def feasible(x, y):
        return all(p * x + q * y <= r for p, q, r in allL)

    best = None
    for i in range(len(allL)):
        p1, q1, r1 = allL[i]
        for j in range(i + 1, len(allL)):
            p2, q2, r2 = allL[j]
            det = p1 * q2 - q1 * p2
            if det == 0:
                continue
            x = (r1 * q2 - r2 * q1) / det
            y = (p1 * r2 - p2 * r1) / det
            if not feasible(x, y):
                continue
            key = (c[0] * x + c[1] * y, -x, -y)
            if best is None or key > best[0]:
                best = (key, x, y)
    if best is None:
        return INFEASIBLE, None, None
    _, x, y = best
    if abs(x) == R or abs(y) == R:
        return UNBOUNDED, None, None
    return OPTIMAL, x, y


def brute_force_batch(batch):
    res = []
    for k in range(batch.offsets.shape[0] - 1):
        s, e = int(batch.offsets[k]), int(batch.offsets[k + 1])
        res.append(brute_force(batch.ax[s:e], batch.ay[s:e], batch.b[s:e], batch.cx[k], batch.cy[k]))
    return res


# ---------------------------------------------------------------------------
# Three dimensions: maximize c.x over R^3 subject to a_i.x <= b_i and
# |x_k| <= M; the lexicographically smallest maximiser (smallest x, then y,
# then z).  UNBOUNDED means the optimum lies on a face of the box.
# ---------------------------------------------------------------------------

def _load3():
    global _lib3
    if _lib3 is None:
        if not os.path.exists(_LIB3) or os.path.getmtime(_LIB3) < os.path.getmtime(_SRC3):
            build(force=False)
        lib = ctypes.CDLL(_LIB3)
        f = lib.rgb_oracle3_solve_range
        P = ctypes.c_void_p
        f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64] + [P] * 8 + [ctypes.c_double] + [P] * 3
        f.restype = ctypes.c_int
        _lib3 = lib
    return _lib3


def solve3(batch, threads: int | None = None, lp_begin: int = 0, lp_end: int | None = None):
    """Solve LPs [lp_begin, lp_end) of a ``gen3.Batch3``.  Returns a dict with
    x (B, 3) float64, status (int32) and def (B, 3) int32 (the planes of the
    optimal vertex: rows 0..m-1, box faces -1..-6), plus the thread count.
    LPs are split over threads by equal sum of m^4 (the enumeration's cost)."""
    lib = _load3()
    offsets = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    arrs = [np.ascontiguousarray(getattr(batch, f), dtype=np.float32) for f in ("ax", "ay", "az", "b", "cx", "cy", "cz")]
    B = offsets.shape[0] - 1
    if lp_end is None:
        lp_end = B
    out = {"x": np.full((B, 3), np.nan), "status": np.full(B, INVALID, dtype=np.int32),
           "def": np.full((B, 3), -100, dtype=np.int32)}
    if threads is None:
        threads = max(1, len(os.sched_getaffinity(0)))
    n = lp_end - lp_begin
    if n <= 0:
        out["threads"] = 0
        return out
    threads = max(1, min(threads, n))
    m = np.diff(offsets[lp_begin:lp_end + 1]).astype(np.float64) + 6.0
    work = np.concatenate([[0.0], np.cumsum(m ** 4)])
    cuts = np.searchsorted(work, np.linspace(0, work[-1], threads + 1)[1:-1]) + lp_begin
    bounds = [lp_begin] + sorted(set(int(c) for c in cuts if lp_begin < c < lp_end)) + [lp_end]
    N = int(batch.b.shape[0])
    args = [_ptr(offsets)] + [_ptr(a) for a in arrs] + [ctypes.c_double(float(batch.box))] + \
        [_ptr(out["x"]), _ptr(out["status"]), _ptr(out["def"])]

    def run(s, e):
        if e > s:
            lib.rgb_oracle3_solve_range(s, e, N, *args)

    ths = [threading.Thread(target=run, args=(bounds[i], bounds[i + 1])) for i in range(len(bounds) - 1)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    out["threads"] = len(ths)
    return out


def _det3(p, q, r):
    return (p[0] * (q[1] * r[2] - q[2] * r[1]) - p[1] * (q[0] * r[2] - q[2] * r[0])
            + p[2] * (q[0] * r[1] - q[1] * r[0]))


def brute_force3(ax, ay, az, b, c, M):
    """Exact rational vertex enumeration of one 3D LP inside the box |x_k| <= M.
    Returns (status, (x, y, z) as Fractions or None)."""
    if not all(np.isfinite(v) for v in list(ax) + list(ay) + list(az) + list(b) + list(c)) or \
            not (np.isfinite(M) and M > 0):
        return INVALID, None
    Mf = _frac(M)
    rows = []
    for p, q, r, s in zip(ax, ay, az, b):
        a = (_frac(p), _frac(q), _frac(r))
        if a == (0, 0, 0):
            if _frac(s) < 0:
                return INFEASIBLE, None
            continue
        rows.append((a, _frac(s)))
    for k in range(3):
        for sgn in (1, -1):
            e = [Fraction(0)] * 3
            e[k] = Fraction(sgn)
            rows.append((tuple(e), Mf))
    cf = tuple(_frac(v) for v in c)
    best = None
    n = len(rows)
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n):
                A, B, C = rows[i][0], rows[j][0], rows[k][0]
                D = _det3(A, B, C)
                if D == 0:
                    continue
                rhs = (rows[i][1], rows[j][1], rows[k][1])
                v = []
                for col in range(3):
                    cols = [list(A), list(B), list(C)]
                    for t in range(3):
                        cols[t][col] = rhs[t]
                    v.append(_det3(*cols) / D)
                key = (sum(ci * vi for ci, vi in zip(cf, v)), -v[0], -v[1], -v[2])
                if best is not None and key <= best[0]:
                    continue
                if all(sum(ai * vi for ai, vi in zip(a, v)) <= bb for a, bb in rows):
                    best = (key, v)
    if best is None:
        return INFEASIBLE, None
    v = best[1]
    return (UNBOUNDED if max(abs(t) for t in v) == Mf else OPTIMAL), tuple(v)


def brute_force3_batch(batch):
    return [brute_force3(*batch.lp(k)[:4], batch.lp(k)[4], batch.box) for k in range(batch.num_lps)]


# ---------------------------------------------------------------------------

def _loadn():
    global _libn
    if _libn is None:
        if not os.path.exists(_LIBN) or os.path.getmtime(_LIBN) < os.path.getmtime(_SRCN):
            build(force=False)
        lib = ctypes.CDLL(_LIBN)
        f = lib.rgb_oraclen_solve_range
        P = ctypes.c_void_p
        f.argtypes = [ctypes.c_int] + [ctypes.c_int64] * 4 + [P] * 4 + [ctypes.c_double] + [P] * 3
        f.restype = ctypes.c_int
        _libn = lib
    return _libn


def solve_n(batch, threads: int | None = None, lp_begin: int = 0, lp_end: int | None = None):
    """Solve LPs [lp_begin, lp_end) of a ``genn.BatchN`` (n = batch.dim).
    Returns a dict with x (B, n) float64, status (int32) and def (B, n) int32
    (the hyperplanes of the optimal vertex: rows 0..m-1, box faces -1..-2n),
    plus the thread count.  LPs are split over threads by equal sum of
    (m + 2n)^n (the enumeration's cost)."""
    lib = _loadn()
    n = int(batch.a.shape[0])
    offsets = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    a = np.ascontiguousarray(batch.a, dtype=np.float32)
    b = np.ascontiguousarray(batch.b, dtype=np.float32)
    c = np.ascontiguousarray(batch.c, dtype=np.float32)
    B = offsets.shape[0] - 1
    if lp_end is None:
        lp_end = B
    out = {"x": np.full((B, n), np.nan), "status": np.full(B, INVALID, dtype=np.int32),
           "def": np.full((B, n), -100, dtype=np.int32)}
    if threads is None:
        threads = max(1, len(os.sched_getaffinity(0)))
    cnt = lp_end - lp_begin
    if cnt <= 0:
        out["threads"] = 0
        return out
    threads = max(1, min(threads, cnt))
    m = np.diff(offsets[lp_begin:lp_end + 1]).astype(np.float64) + 2.0 * n
    work = np.concatenate([[0.0], np.cumsum(m ** n)])
    cuts = np.searchsorted(work, np.linspace(0, work[-1], threads + 1)[1:-1]) + lp_begin
    bounds = [lp_begin] + sorted(set(int(t) for t in cuts if lp_begin < t < lp_end)) + [lp_end]
    N = int(b.shape[0])
    args = [_ptr(offsets), _ptr(a), _ptr(b), _ptr(c), ctypes.c_double(float(batch.box)),
            _ptr(out["x"]), _ptr(out["status"]), _ptr(out["def"])]
    rc = []

    def run(s, e):
        if e > s:
            rc.append(lib.rgb_oraclen_solve_range(n, s, e, B, N, *args))

    ths = [threading.Thread(target=run, args=(bounds[i], bounds[i + 1])) for i in range(len(bounds) - 1)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    if any(r != 0 for r in rc):
        raise ValueError(f"dimension {n} is outside 1..6")
    out["threads"] = len(ths)
    return out


def _int_row(vals):
    """Fractions scaled by a positive integer into integers (a row's
    constraint, or the objective's argmax, does not change)."""
    from math import lcm
    den = 1
    for v in vals:
        den = lcm(den, v.denominator)
    return [int(v * den) for v in vals]


def _solve_int(A, r):
    """Solve the integer system A v = r exactly by fraction-free Gauss-Jordan
    elimination (every division is exact).  Returns (N, D) with v = N / D and
    D > 0, or None when the system is singular."""
    n = len(A)
    M = [list(A[i]) + [r[i]] for i in range(n)]
    prev = 1
    for k in range(n):
        p = next((i for i in range(k, n) if M[i][k] != 0), None)
        if p is None:
            return None
        M[k], M[p] = M[p], M[k]
        pk = M[k][k]
        for i in range(n):
            if i == k:
                continue
            mik = M[i][k]
            M[i] = [(pk * M[i][j] - mik * M[k][j]) // prev if j != k else 0 for j in range(n + 1)]
        prev = pk
    D = M[0][0]
    N = [M[i][n] for i in range(n)]
    if D < 0:
        D, N = -D, [-t for t in N]
    return N, D


def brute_force_n(a, b, c, M):
    """Exact rational vertex enumeration of one LP in n dimensions inside the
    box |x_k| <= M: a is (n, m), b (m,), c (n,).  Every row is scaled to
    integers and each vertex is solved in exact integer arithmetic.  Returns
    (status, x as a tuple of Fractions or None)."""
    from itertools import combinations
    a = np.asarray(a)
    n, m = a.shape
    vals = list(a.ravel()) + list(b) + list(c)
    if not all(np.isfinite(v) for v in vals) or not (np.isfinite(M) and M > 0):
        return INVALID, None
    Mf = _frac(M)
    rows = []
    for i in range(m):
        ai = [_frac(a[k, i]) for k in range(n)]
        if all(t == 0 for t in ai):
            if _frac(b[i]) < 0:
                return INFEASIBLE, None
            continue
        r = _int_row(ai + [_frac(b[i])])
        rows.append((r[:n], r[n]))
    for k in range(n):
        for sgn in (1, -1):
            e = [0] * n
            e[k] = sgn * Mf.denominator
            rows.append((e, Mf.numerator))
    cf = _int_row([_frac(v) for v in c])
    best = None  # (c.N, N, D)
    for sub in combinations(range(len(rows)), n):
        sol = _solve_int([rows[i][0] for i in sub], [rows[i][1] for i in sub])
        if sol is None:
            continue
        N, D = sol
        f = sum(ci * t for ci, t in zip(cf, N))
        if best is not None:
            bf, bN, bD = best
            lhs, rhs = f * bD, bf * D
            if lhs < rhs:
                continue
            if lhs == rhs:
                # equal objective: the smaller x_1, then x_2, ... wins
                cmp = next(((t * bD > u * D) - (t * bD < u * D) for t, u in zip(N, bN) if t * bD != u * D), 0)
                if cmp >= 0:
                    continue
        if all(sum(ai * t for ai, t in zip(r, N)) <= bb * D for r, bb in rows):
            best = (f, N, D)
    if best is None:
        return INFEASIBLE, None
    _, N, D = best
    v = tuple(Fraction(t, D) for t in N)
    return (UNBOUNDED if max(abs(t) for t in v) == Mf else OPTIMAL), v


def brute_force_n_batch(batch):
    return [brute_force_n(*batch.lp(k), batch.box) for k in range(batch.num_lps)]
