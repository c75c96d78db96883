"""Seeded synthetic inputs for batched two-dimensional LPs.

This module only draws random numbers and lays them out; it holds none of the
solver's arithmetic, so the FP64 oracle and the HIP path can both take their
inputs from it.

Every LP is ``maximize c.x subject to a_i.x <= b_i`` (Eq. (1)-(2) of the paper)
and a batch is stored CSR-offset SoA: ``offsets`` (int64, B+1), half-plane
arrays ``ax, ay, b`` (float32, offsets[B]) and objectives ``cx, cy`` (float32,
B).  The solver keeps the input order, so the random constraint order that
Seidel's expected O(m) bound needs (Sec. 2.1) is drawn here.

The paper fills each batch with copies of a single random feasible LP (Sec. 4);
these generators draw a distinct LP per slot instead, so per-LP work is uneven
the way the paper's work-unit design expects (Sec. 3).

Shuffle: the random rows of an LP are i.i.d., hence exchangeable, so a uniform
shuffle of "random rows + k special rows" has the same law as inserting the k
special rows one after the other at uniform positions.  That is what
``_assemble`` does, in O(N) and vectorised.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

SEED_ROOT = 20190213

# per-LP construction tags (diagnostic only; never read by a solver)
KIND_BOXED = 0        # random half-planes containing the unit disk, plus the |x|,|y| <= box rows
KIND_INFEASIBLE = 1   # boxed LP plus the pair a*.x <= -3, -a*.x <= -3
KIND_UNBOUNDED = 2    # normals in a half circle, no box, c inside the recession cone's dual
KIND_CROWD = 3        # neighbour half-planes plus a 16-gon speed limit
KIND_OTHER = 4


@dataclasses.dataclass
class Batch:
    offsets: np.ndarray
    ax: np.ndarray
    ay: np.ndarray
    b: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    kind: np.ndarray
    name: str = ""

    @property
    def num_lps(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def num_constraints(self) -> int:
        return int(self.offsets[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def algorithmic_bytes(self) -> int:
        """One read of (a_x, a_y, b) per half-plane plus, per LP, its offset,
        objective and the (x, y, status) it writes: 12 B * N + 28 B * B."""
        return 12 * self.num_constraints + 28 * self.num_lps

    def lp(self, k: int):
        s, e = int(self.offsets[k]), int(self.offsets[k + 1])
        return (self.ax[s:e], self.ay[s:e], self.b[s:e], float(self.cx[k]), float(self.cy[k]))

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx, dtype=np.int64)
        sizes = self.sizes()[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(sizes, out=offs[1:])
        starts = self.offsets[idx]
        gather = (np.repeat(starts - offs[:-1], sizes) + np.arange(offs[-1], dtype=np.int64))
        return Batch(offs, self.ax[gather], self.ay[gather], self.b[gather],
                     self.cx[idx], self.cy[idx], self.kind[idx], self.name + "[subset]")

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.offsets, self.ax, self.ay, self.b, self.cx, self.cy):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()


def concat(batches, name="concat") -> Batch:
    sizes = np.concatenate([bt.sizes() for bt in batches])
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    cat = lambda f: np.concatenate([getattr(bt, f) for bt in batches])
    return Batch(offs, cat("ax"), cat("ay"), cat("b"), cat("cx"), cat("cy"), cat("kind"), name)


def rng_for(*keys) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, *keys])))


def _box_rows(box: float):
    return np.array([[1.0, 0.0, box], [-1.0, 0.0, box], [0.0, 1.0, box], [0.0, -1.0, box]])


def _assemble(rng, n_rand, theta_lo, theta_w, specials, n_spec, c_angle, kind, name,
              b_lo=1.0, b_hi=2.0) -> Batch:
    """Lay out B LPs.  LP k gets n_rand[k] random rows with normal angle
    theta_lo[k] + theta_w[k]*U[0,1) and offset U[b_lo, b_hi), plus the first
    n_spec[k] rows of specials[k] inserted at uniform positions."""
    B = n_rand.shape[0]
    n_rand = n_rand.astype(np.int64)
    n_spec = n_spec.astype(np.int64)
    sizes = n_rand + n_spec
    offsets = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    N = int(offsets[-1])

    # random rows, LP-major, in the order they will appear
    lp_of_row = np.repeat(np.arange(B, dtype=np.int64), n_rand)
    theta = theta_lo[lp_of_row] + theta_w[lp_of_row] * rng.random(lp_of_row.shape[0])
    rax = np.cos(theta).astype(np.float32)
    ray = np.sin(theta).astype(np.float32)
    del theta
    rb = (b_lo + (b_hi - b_lo) * rng.random(lp_of_row.shape[0])).astype(np.float32)
    del lp_of_row

    ax = np.empty(N, dtype=np.float32)
    ay = np.empty(N, dtype=np.float32)
    bb = np.empty(N, dtype=np.float32)
    K = specials.shape[1] if specials.ndim == 3 else 0
    if K == 0 or int(n_spec.max(initial=0)) == 0:
        ax[:], ay[:], bb[:] = rax, ray, rb
    else:
        pos = np.zeros((B, K), dtype=np.int64)
        for j in range(K):
            active = j < n_spec
            pj = np.floor(rng.random(B) * (n_rand + j + 1)).astype(np.int64)
            pj = np.minimum(pj, n_rand + j)
            shift = (pos[:, :j] >= pj[:, None]) & active[:, None]
            pos[:, :j] += shift
            pos[:, j] = np.where(active, pj, 0)
        valid = np.arange(K)[None, :] < n_spec[:, None]
        gidx = (offsets[:-1, None] + pos)[valid]
        is_spec = np.zeros(N, dtype=bool)
        is_spec[gidx] = True
        free = np.flatnonzero(~is_spec)
        ax[free], ay[free], bb[free] = rax, ray, rb
        sp = specials[valid]
        ax[gidx] = sp[:, 0].astype(np.float32)
        ay[gidx] = sp[:, 1].astype(np.float32)
        bb[gidx] = sp[:, 2].astype(np.float32)
    cx = np.cos(c_angle).astype(np.float32)
    cy = np.sin(c_angle).astype(np.float32)
    return Batch(offsets, ax, ay, bb, cx, cy, kind.astype(np.int8), name)


def _mixed(rng, m_rand, infeasible_frac, unbounded_frac, box, name, exact_counts=True) -> Batch:
    """Boxed random LPs with a share made infeasible (antiparallel pair with a
    gap) and a share made unbounded (no box, normals in a half circle, c within
    pi/3 of a recession direction)."""
    B = m_rand.shape[0]
    kind = np.full(B, KIND_BOXED, dtype=np.int64)
    if exact_counts:
        perm = rng.permutation(B)
        n_inf = int(round(infeasible_frac * B))
        n_unb = int(round(unbounded_frac * B))
        kind[perm[:n_inf]] = KIND_INFEASIBLE
        kind[perm[n_inf:n_inf + n_unb]] = KIND_UNBOUNDED
    else:
        u = rng.random(B)
        kind[u < infeasible_frac] = KIND_INFEASIBLE
        kind[(u >= infeasible_frac) & (u < infeasible_frac + unbounded_frac)] = KIND_UNBOUNDED

    theta_lo = np.zeros(B)
    theta_w = np.full(B, 2.0 * math.pi)
    c_angle = rng.random(B) * 2.0 * math.pi
    unb = kind == KIND_UNBOUNDED
    th0 = rng.random(B) * 2.0 * math.pi
    theta_lo[unb] = th0[unb]
    theta_w[unb] = math.pi
    c_angle[unb] = th0[unb] - 0.5 * math.pi + (rng.random(int(unb.sum())) * 2.0 - 1.0) * (math.pi / 3.0)

    specials = np.zeros((B, 6, 3))
    n_spec = np.zeros(B, dtype=np.int64)
    boxed = kind != KIND_UNBOUNDED
    specials[boxed, :4, :] = _box_rows(box)
    n_spec[boxed] = 4
    inf = kind == KIND_INFEASIBLE
    ts = rng.random(B) * 2.0 * math.pi
    asx = np.cos(ts).astype(np.float32).astype(np.float64)
    asy = np.sin(ts).astype(np.float32).astype(np.float64)
    specials[inf, 4, :] = np.stack([asx[inf], asy[inf], np.full(int(inf.sum()), -3.0)], axis=1)
    specials[inf, 5, :] = np.stack([-asx[inf], -asy[inf], np.full(int(inf.sum()), -3.0)], axis=1)
    n_spec[inf] = 6
    return _assemble(rng, m_rand, theta_lo, theta_w, specials, n_spec, c_angle, kind, name)


def uniform_batch(num_lps: int, m: int, seed: int = 0, infeasible_frac=0.05, unbounded_frac=0.02,
                  box=1e6, name=None) -> Batch:
    """num_lps LPs with m random half-planes each (unit normals at uniform
    angles, offsets U[1,2]) plus the 4 box rows; the infeasible share gets 2
    more rows, the unbounded share drops the box."""
    rng = rng_for(1, num_lps, m, seed)
    return _mixed(rng, np.full(num_lps, m, dtype=np.int64), infeasible_frac, unbounded_frac, box,
                  name or f"uniform_{num_lps}x{m}")


def uneven_batch(num_lps: int, m_lo: int = 8, m_hi: int = 8192, seed: int = 0, infeasible_frac=0.05,
                 unbounded_frac=0.02, box=1e6, name=None) -> Batch:
    """Random-row counts log-uniform in [m_lo, m_hi]."""
    rng = rng_for(2, num_lps, m_lo, m_hi, seed)
    m = np.floor(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi + 1), num_lps))).astype(np.int64)
    m = np.clip(m, m_lo, m_hi)
    return _mixed(rng, m, infeasible_frac, unbounded_frac, box, name or f"uneven_{num_lps}_{m_lo}_{m_hi}")


def crowd_batch(num_agents: int = 262144, seed: int = 0, density: float = 1.0, k_lo: int = 8,
                k_hi: int = 64, radius: float = 0.3, vmax: float = 1.0, n_disc: int = 16,
                name=None) -> Batch:
    """Velocity-space LPs shaped like crowd collision avoidance: agents uniform
    in a square at the given density; agent i gets one half-plane per nearest
    neighbour (k_i ~ U{k_lo..k_hi}), normal = unit vector towards the
    neighbour, offset 0.5*(distance - radius); the speed disc |v| <= vmax is
    replaced by n_disc tangent half-planes; c is a unit preferred velocity."""
    from scipy.spatial import cKDTree

    rng = rng_for(4, num_agents, seed)
    side = math.sqrt(num_agents / density)
    pos = rng.random((num_agents, 2)) * side
    k = rng.integers(k_lo, k_hi + 1, num_agents)
    tree = cKDTree(pos)
    _, nbr = tree.query(pos, k=k_hi + 1)
    nbr = nbr[:, 1:]
    sel = np.arange(k_hi)[None, :] < k[:, None]
    src = np.repeat(np.arange(num_agents), k)
    dst = nbr[sel]
    d = pos[dst] - pos[src]
    dist = np.hypot(d[:, 0], d[:, 1])
    zero = dist == 0.0
    dist_safe = np.where(zero, 1.0, dist)
    nx = np.where(zero, 1.0, d[:, 0] / dist_safe)
    ny = np.where(zero, 0.0, d[:, 1] / dist_safe)
    off = 0.5 * (dist - radius)

    # neighbour rows are exchangeable only approximately (sorted by distance), so
    # shuffle every row of the LP with random keys inside each segment
    n_rows = k + n_disc
    offsets = np.zeros(num_agents + 1, dtype=np.int64)
    np.cumsum(n_rows, out=offsets[1:])
    N = int(offsets[-1])
    lp = np.repeat(np.arange(num_agents, dtype=np.int64), n_rows)
    local = np.arange(N, dtype=np.int64) - offsets[lp]
    is_nbr = local < np.repeat(k, n_rows)
    rows = np.empty((N, 3))
    rows[is_nbr, 0], rows[is_nbr, 1], rows[is_nbr, 2] = nx, ny, off
    disc = np.arange(n_disc) * (2.0 * math.pi / n_disc)
    j = (local[~is_nbr] - np.repeat(k, n_rows)[~is_nbr])
    rows[~is_nbr, 0] = np.cos(disc)[j]
    rows[~is_nbr, 1] = np.sin(disc)[j]
    rows[~is_nbr, 2] = vmax
    order = np.lexsort((rng.random(N), lp))
    rows = rows[order]
    c_angle = rng.random(num_agents) * 2.0 * math.pi
    return Batch(offsets, rows[:, 0].astype(np.float32), rows[:, 1].astype(np.float32),
                 rows[:, 2].astype(np.float32), np.cos(c_angle).astype(np.float32),
                 np.sin(c_angle).astype(np.float32), np.full(num_agents, KIND_CROWD, np.int8),
                 name or f"crowd_{num_agents}")


def served_request(rng: np.random.Generator, max_lps=4096, m_lo=16, m_hi=2048, infeasible_frac=0.05,
                   unbounded_frac=0.02, box=1e6) -> Batch:
    """One request of the served stream: n ~ floor(logU[1, max_lps]) LPs with
    random-row counts log-uniform in [m_lo, m_hi], same mix as the batches."""
    n = int(min(max_lps, max(1, math.floor(math.exp(rng.uniform(0.0, math.log(max_lps + 1)))))))
    m = np.floor(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi + 1), n))).astype(np.int64)
    m = np.clip(m, m_lo, m_hi)
    return _mixed(rng, m, infeasible_frac, unbounded_frac, box, "request", exact_counts=False)


def poisson_arrivals(rng: np.random.Generator, n: int, rate_per_s: float) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


def tiny_integer_batch(num_lps: int, m_max: int = 8, K: int = 4, seed: int = 0, m_min: int = 0,
                       zero_c_frac: float = 0.1, boxed: bool = False) -> Batch:
    """Small LPs with integer coefficients in [-K, K] (exact in fp32), so that
    degenerate cases (parallel and coincident lines, concurrent lines, zero
    normals, c = 0, single-point regions) appear often.  ``boxed`` inserts the
    rows |x|, |y| <= K at random positions, which makes most LPs bounded."""
    if boxed:
        base = tiny_integer_batch(num_lps, m_max, K, seed, m_min, zero_c_frac, boxed=False)
        rng = rng_for(9, num_lps, m_max, K, seed)
        sizes = base.sizes()
        specials = np.broadcast_to(_box_rows(float(K)), (num_lps, 4, 3)).copy()
        out = _assemble_fixed(rng, base, specials)
        out.name = f"tiny_int_boxed_{num_lps}"
        return out
    rng = rng_for(7, num_lps, m_max, K, seed)
    m = rng.integers(m_min, m_max + 1, num_lps)
    offsets = np.zeros(num_lps + 1, dtype=np.int64)
    np.cumsum(m, out=offsets[1:])
    N = int(offsets[-1])
    ax = rng.integers(-K, K + 1, N).astype(np.float32)
    ay = rng.integers(-K, K + 1, N).astype(np.float32)
    b = rng.integers(-K, K + 1, N).astype(np.float32)
    cx = rng.integers(-K, K + 1, num_lps).astype(np.float32)
    cy = rng.integers(-K, K + 1, num_lps).astype(np.float32)
    z = rng.random(num_lps) < zero_c_frac
    cx[z] = 0.0
    cy[z] = 0.0
    return Batch(offsets, ax, ay, b, cx, cy, np.full(num_lps, KIND_OTHER, np.int8), f"tiny_int_{num_lps}")


def _assemble_fixed(rng, base: Batch, specials: np.ndarray) -> Batch:
    """Insert the rows specials[k] of each LP k at uniform positions among the
    existing rows of ``base`` (which keep their order)."""
    B, K, _ = specials.shape
    n_rand = base.sizes()
    pos = np.zeros((B, K), dtype=np.int64)
    for j in range(K):
        pj = np.minimum(np.floor(rng.random(B) * (n_rand + j + 1)).astype(np.int64), n_rand + j)
        pos[:, :j] += pos[:, :j] >= pj[:, None]
        pos[:, j] = pj
    sizes = n_rand + K
    offsets = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    N = int(offsets[-1])
    gidx = (offsets[:-1, None] + pos).ravel()
    is_spec = np.zeros(N, dtype=bool)
    is_spec[gidx] = True
    free = np.flatnonzero(~is_spec)
    ax = np.empty(N, np.float32)
    ay = np.empty(N, np.float32)
    bb = np.empty(N, np.float32)
    ax[free], ay[free], bb[free] = base.ax, base.ay, base.b
    sp = specials.reshape(-1, 3)
    ax[gidx], ay[gidx], bb[gidx] = sp[:, 0], sp[:, 1], sp[:, 2]
    return Batch(offsets, ax, ay, bb, base.cx.copy(), base.cy.copy(), base.kind.copy(), base.name)


def tiny_random_batch(num_lps: int, m_max: int = 40, seed: int = 0, m_min: int = 0) -> Batch:
    """Small LPs with continuous coefficients: normals at uniform angles with
    random length in [0.5, 2], offsets U[-0.5, 2], unit objective.  Roughly a
    third of them end up infeasible and some unbounded."""
    rng = rng_for(8, num_lps, m_max, seed)
    m = rng.integers(m_min, m_max + 1, num_lps)
    offsets = np.zeros(num_lps + 1, dtype=np.int64)
    np.cumsum(m, out=offsets[1:])
    N = int(offsets[-1])
    th = rng.random(N) * 2.0 * math.pi
    r = 0.5 + 1.5 * rng.random(N)
    ax = (r * np.cos(th)).astype(np.float32)
    ay = (r * np.sin(th)).astype(np.float32)
    b = (-0.5 + 2.5 * rng.random(N)).astype(np.float32)
    ca = rng.random(num_lps) * 2.0 * math.pi
    return Batch(offsets, ax, ay, b, np.cos(ca).astype(np.float32), np.sin(ca).astype(np.float32),
                 np.full(num_lps, KIND_OTHER, np.int8), f"tiny_rand_{num_lps}")


# Named workloads.  ``scale`` shrinks the LP count for parity tests the oracle
# finishes in seconds; scale=1 is the full size.
def device_disk_batch(num_lps: int, m: int, seed: int, device="cuda"):
    """A batch built directly in device memory (for sizes the host should not
    generate): LP k has rows m*k .. m*k+m-1 with unit normals (cos t, sin t),
    t ~ U[0, 2 pi), offsets b ~ U[1, 2] (so every LP contains the unit disk)
    and a random unit objective.  Seeded torch generator on the device;
    returns (offsets, ax, ay, b, cx, cy) tensors."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    n = num_lps * m
    t = torch.rand(n, generator=g, device=device) * (2.0 * np.pi)
    ax = torch.cos(t)
    ay = torch.sin(t)
    del t
    b = torch.rand(n, generator=g, device=device) + 1.0
    u = torch.rand(num_lps, generator=g, device=device) * (2.0 * np.pi)
    cx, cy = torch.cos(u), torch.sin(u)
    offsets = torch.arange(num_lps + 1, device=device, dtype=torch.int64) * m
    return offsets, ax, ay, b, cx, cy


def host_subset(offsets, ax, ay, b, cx, cy, idx) -> Batch:
    """Copy the LPs `idx` of a device batch (tensors as from device_disk_batch)
    into a host Batch."""
    import torch
    idx = np.asarray(idx, dtype=np.int64)
    lo = offsets[torch.as_tensor(idx, device=offsets.device)].cpu().numpy()
    hi = offsets[torch.as_tensor(idx + 1, device=offsets.device)].cpu().numpy()
    sizes = hi - lo
    out_offs = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(sizes, out=out_offs[1:])
    gather = np.repeat(lo - out_offs[:-1], sizes) + np.arange(out_offs[-1], dtype=np.int64)
    gi = torch.as_tensor(gather, device=ax.device)
    pick = lambda t: t[gi].cpu().numpy().astype(np.float32)
    ti = torch.as_tensor(idx, device=cx.device)
    return Batch(out_offs, pick(ax), pick(ay), pick(b), cx[ti].cpu().numpy().astype(np.float32),
                 cy[ti].cpu().numpy().astype(np.float32), np.full(len(idx), KIND_OTHER, np.int8), "device[subset]")


CONFIGS = {
    "plain": dict(kind="uniform", num_lps=1024, m=64, infeasible_frac=0.0, unbounded_frac=0.0),
    "uniform": dict(kind="uniform", num_lps=131072, m=256),
    "uneven": dict(kind="uneven", num_lps=200000, m_lo=8, m_hi=8192),
    "crowd": dict(kind="crowd", num_agents=262144),
}


def make_config(name: str, seed: int = 0, scale: float = 1.0) -> Batch:
    cfg = dict(CONFIGS[name])
    kind = cfg.pop("kind")
    if kind == "uniform":
        n = max(1, int(round(cfg.pop("num_lps") * scale)))
        return uniform_batch(n, seed=seed, name=name, **cfg)
    if kind == "uneven":
        n = max(1, int(round(cfg.pop("num_lps") * scale)))
        return uneven_batch(n, seed=seed, name=name, **cfg)
    if kind == "crowd":
        n = max(64, int(round(cfg.pop("num_agents") * scale)))
        return crowd_batch(n, seed=seed, name=name, **cfg)
    raise KeyError(name)
