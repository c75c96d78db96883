"""Memory-row model of the binned kernel on a sample of the uneven recipe.

    python -m paper_1902_04995_amd.traffic_model [--lps 2000] [--seed 7]

Counts, per size class, the rows the binned launch reads from memory for
each LP, given the order in which Seidel's method meets violated rows (Sec.
2.1): every row once as the scan passes it; for a violation at row v, the 1D
LP (Eq. (3)-(4)) re-reads rows [rg, cs) from memory, where cs is the start of
the scan chunk holding v (the chunk's own rows are in registers) and rg the
LP's share of the wave's LDS cache (its leading rows); and, for a kernel
without the recorded bound steps, one more pass over rows [0, l) at the end,
l the last violated row, to find the vertex's second defining row.  The
violation order comes from a plain FP64 replay of the method on the sample
(a model for counting, not a solver: its ties and degenerate cases are
decided loosely).  Prints the traffic relative to one read of every row,
with and without the end-of-LP pass.
"""
from __future__ import annotations

import argparse
import math

import numpy as np

# lanes per LP (log2) by size class ceil(log2 m), as the autotuner picks them
# for the uneven batch; scan rows per lane by width; LDS rows per wave
LOG2_LANES = [2, 2, 2, 2, 2, 3, 3, 4, 4, 5, 6, 6, 6, 6, 6, 6]
CACHE_ROWS = 448


def scan_rows(lg: int) -> int:
    return 4 if lg >= 6 else 2 if lg >= 3 else 1


def violations(ax, ay, b, c):
    """Rows at which the incremental method meets a violated row, and whether
    it ended infeasible.  Starts from a point far along c (the box corner)."""
    A = np.stack([ax, ay], 1).astype(np.float64)
    b = b.astype(np.float64)
    c = c.astype(np.float64)
    n = np.linalg.norm(c)
    x = c / n * 1e9 if n > 0 else np.full(2, 1e9)
    viol = A @ x - b
    out = []
    for i in range(len(b)):
        if viol[i] <= 1e-9 * max(1.0, abs(b[i])):
            continue
        out.append(i)
        a = A[i]
        if not a.any():
            return out, True
        p0 = a * b[i] / (a @ a)
        d = np.array([-a[1], a[0]])
        s = A[:i] @ d
        r = b[:i] - A[:i] @ p0
        pos, neg = s > 1e-15, s < -1e-15
        hi = np.min(r[pos] / s[pos]) if pos.any() else np.inf
        lo = np.max(r[neg] / s[neg]) if neg.any() else -np.inf
        if np.any((~pos & ~neg) & (r < 0)) or lo > hi:
            return out, True
        t = hi if c @ d > 0 else lo
        if not np.isfinite(t):
            t = 1e9 if c @ d > 0 else -1e9
        x = p0 + t * d
        viol = A @ x - b
    return out, False


def model(bt):
    """Rows read per size class: (first reads, 1D-LP re-reads, end-of-LP pass)."""
    per = {}
    for k in range(bt.num_lps):
        s, e = int(bt.offsets[k]), int(bt.offsets[k + 1])
        m = e - s
        cls = max(0, math.ceil(math.log2(max(m, 1))))
        lg = LOG2_LANES[min(cls, 15)]
        chunk = scan_rows(lg) << lg
        rg = CACHE_ROWS >> (6 - lg)
        vs, dead = violations(bt.ax[s:e], bt.ay[s:e], bt.b[s:e], np.array([bt.cx[k], bt.cy[k]]))
        re = sum(max(0, (v // chunk) * chunk - rg) for v in vs)
        fin = vs[-1] if vs and not dead else 0
        acc = per.setdefault(min(cls, 13), [0, 0, 0])
        acc[0] += m
        acc[1] += re
        acc[2] += fin
    return per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lps", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    from paper_1902_04995_amd import gen
    bt = gen.uneven_batch(args.lps, seed=args.seed)
    per = model(bt)
    tot = np.sum(list(per.values()), axis=0)
    print(f"{bt.num_lps} LPs, {tot[0]} rows: traffic / one read = {(tot[0] + tot[1]) / tot[0]:.3f} "
          f"(with the end-of-LP pass {(tot.sum()) / tot[0]:.3f})")
    for cls in sorted(per):
        f, r, e = per[cls]
        print(f"  class {cls:2d} (rows <= {1 << cls}): {f} rows, x {(f + r) / f:.3f} (with the pass x {(f + r + e) / f:.3f})")


if __name__ == "__main__":
    main()
