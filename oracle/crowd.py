"""TEST INFRASTRUCTURE ONLY: CPU reference of one crowd time step.

Only ``tests/`` and ``bench.py``'s CPU legs may import this module.  It shares
no code with the HIP path; it restates the step from its definition:

  1. neighbours: agent i's k_i nearest other agents, ordered by the FP32
     squared distance dx*dx + dy*dy (dx, dy FP32 differences), then by index;
  2. LP rows: per neighbour j the half-plane n.v <= (d - radius)/2, n the unit
     vector from i to j (FP32: d = sqrt(dx*dx + dy*dy), n = (dx/d, dy/d), or
     (1, 0) when d = 0), then the speed disc |v| <= vmax as n_disc half-planes
     with normals (cos, sin) of 2 pi q / n_disc rounded from double;
  3. row order: row t of agent i at step s has key
     splitmix64_nth(seed, (s << 40) + (i << 8) + t + 1); rows are sorted by
     the key with its low 7 bits replaced by t;
  4. the LPs are solved by the FP64 oracle (objective = preferred velocity);
  5. v = x* where OPTIMAL, else 0; p += dt v in FP32, clamped to the bounds.

All FP32 arithmetic uses numpy float32 (IEEE, no fused operations), in the
order written above.  The FP32 squared distances decide the neighbour order,
so they are computed exactly as stated, not in FP64.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_nth(seed, n):
    """n-th output (n >= 1, numpy uint64 array) of SplitMix64 seeded with
    `seed`: the state after n steps is seed + n * golden, and the output is the
    published mixing function of that state."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.asarray(n, dtype=np.uint64) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed, count):
    """The first `count` outputs of SplitMix64 as the sequential generator
    (state += golden, then mix): used to pin splitmix64_nth."""
    mask = (1 << 64) - 1
    state, out = int(seed) & mask, []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def sq_dist32(px, py, i, j):
    """FP32 squared distances from agent(s) i to agent(s) j."""
    dx = px[j] - px[i]
    dy = py[j] - py[i]
    return dx * dx + dy * dy


def knn_brute(px, py, k):
    """Exact neighbour lists by brute force over all pairs (small crowds)."""
    n = px.shape[0]
    out = []
    idx = np.arange(n)
    for i in range(n):
        d2 = sq_dist32(px, py, np.full(n, i), idx)
        keys = [(float(d2[j]), j) for j in range(n) if j != i]
        keys.sort()
        out.append([j for _, j in keys[: int(k[i])]])
    return out


def knn(px, py, k, extra=24, agents=None):
    """Exact neighbour lists (of `agents`, default all): candidates from a
    KD-tree in FP64 (the k+extra nearest), then the exact FP32 order on them.
    A candidate outside the FP64 top k+extra would need more than `extra`
    agents within FP32 rounding of the k-th distance."""
    from scipy.spatial import cKDTree

    n = px.shape[0]
    agents = np.arange(n) if agents is None else np.asarray(agents)
    kmax = int(np.max(np.asarray(k)[agents]))
    q = min(n, kmax + extra + 1)
    tree = cKDTree(np.stack([px.astype(np.float64), py.astype(np.float64)], axis=1))
    _, cand = tree.query(np.stack([px[agents], py[agents]], axis=1).astype(np.float64), k=q)
    out = []
    for row, i in enumerate(agents):
        c = cand[row]
        c = c[c != i]
        d2 = sq_dist32(px, py, np.full(c.shape[0], i), c)
        order = np.lexsort((c, d2))
        out.append(c[order[: int(k[i])]].tolist())
    return out


def disc_rows(n_disc, vmax):
    ang = [2.0 * math.pi * q / n_disc for q in range(n_disc)]
    return (np.array([math.cos(a) for a in ang], np.float32), np.array([math.sin(a) for a in ang], np.float32),
            np.float32(vmax))


def agent_rows(px, py, i, nbr, radius, vmax, n_disc, seed, step):
    """Rows (ax, ay, b) of agent i's LP, in the keyed order."""
    cs, sn, vm = disc_rows(n_disc, vmax)
    j = np.asarray(nbr, np.int64)
    dx = px[j] - px[i]
    dy = py[j] - py[i]
    dist = np.sqrt(dx * dx + dy * dy)
    zero = dist == np.float32(0.0)
    safe = np.where(zero, np.float32(1.0), dist)
    rx = np.concatenate([np.where(zero, np.float32(1.0), dx / safe), cs])
    ry = np.concatenate([np.where(zero, np.float32(0.0), dy / safe), sn])
    rb = np.concatenate([np.float32(0.5) * (dist - np.float32(radius)), np.full(n_disc, vm, np.float32)])
    t = np.arange(rx.shape[0], dtype=np.uint64)
    ctr = (np.uint64(step) << np.uint64(40)) + (np.uint64(i) << np.uint64(8)) + t
    keys = (splitmix64_nth(seed, ctr + np.uint64(1)) & ~np.uint64(127)) | t
    order = np.argsort(keys, kind="stable")
    return rx[order].astype(np.float32), ry[order].astype(np.float32), rb[order].astype(np.float32)


def build_rows(px, py, k, nbrs, radius, vmax, n_disc, seed, step):
    """CSR rows (offsets, ax, ay, b) of every agent's LP."""
    n = px.shape[0]
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(np.asarray(k, np.int64) + n_disc, out=offsets[1:])
    ax = np.empty(offsets[-1], np.float32)
    ay = np.empty_like(ax)
    b = np.empty_like(ax)
    for i in range(n):
        o, e = offsets[i], offsets[i + 1]
        ax[o:e], ay[o:e], b[o:e] = agent_rows(px, py, i, nbrs[i], radius, vmax, n_disc, seed, step)
    return offsets, ax, ay, b


def integrate(px, py, vx, vy, status, dt, bounds):
    """p += dt v (v = 0 unless OPTIMAL) in FP32, clamped to the bounds."""
    ok = status == 0
    ux = np.where(ok, vx, np.float32(0.0)).astype(np.float32)
    uy = np.where(ok, vy, np.float32(0.0)).astype(np.float32)
    x = px + np.float32(dt) * ux
    y = py + np.float32(dt) * uy
    x = np.clip(x, np.float32(bounds[0]), np.float32(bounds[2])).astype(np.float32)
    y = np.clip(y, np.float32(bounds[1]), np.float32(bounds[3])).astype(np.float32)
    return x, y, ux, uy
