"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for batched 2D LPs.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP solver.

Contents
  * ``solve``      - serial FP64 Seidel in C (``seidel_oracle.c``), driven over
                     LP ranges by Python threads (ctypes drops the GIL).
  * ``brute_force`` - exact rational vertex enumeration for one small LP; the
                     pin the oracle is checked against.
  * ``build``      - compiles ``seidel_oracle.c`` with gcc.
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
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle.  -ffp-contract=off keeps every product and sum
    rounded as written (no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
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
