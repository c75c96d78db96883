"""Seeded synthetic inputs for batched three-dimensional LPs.

Like ``gen``, this module only draws random numbers and lays them out; it holds
none of the solver's arithmetic, so the oracle and the HIP path both take their
inputs from it.

Every LP is ``maximize c.x subject to a_i.x <= b_i`` over x in R^3 (Eq. (1)-(2)
of the paper with n = 3), inside the box ``|x_k| <= box`` (the bounding rows of
Sec. 2.1, given by the caller instead of stored as rows).  A batch is stored
CSR-offset SoA: ``offsets`` (int64, B+1), plane arrays ``ax, ay, az, b``
(float32) and objectives ``cx, cy, cz`` (float32, B).  The solver keeps the
input order, so the random row order Seidel's expected bound needs is drawn
here.  The paper names higher dimensions as its next step (Sec. 6); it has no
3D workload, so these recipes carry its 2D ones over: random planes tangent to
a sphere around the origin at distance U[1, 2] (the 3D form of the 2D lines),
a share made infeasible by an antiparallel pair with a gap, and a share whose
rows leave a recession direction open (reported as touching the box).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

from .gen import KIND_BOXED, KIND_INFEASIBLE, KIND_OTHER, KIND_UNBOUNDED, rng_for


@dataclasses.dataclass
class Batch3:
    offsets: np.ndarray
    ax: np.ndarray
    ay: np.ndarray
    az: np.ndarray
    b: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    cz: np.ndarray
    kind: np.ndarray
    box: float
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
        """One read of (a_x, a_y, a_z, b) per plane plus, per LP, its offset,
        objective and the (x, y, z, status) it writes: 16 B * N + 36 B * B."""
        return 16 * self.num_constraints + 36 * self.num_lps

    def lp(self, k: int):
        s, e = int(self.offsets[k]), int(self.offsets[k + 1])
        return (self.ax[s:e], self.ay[s:e], self.az[s:e], self.b[s:e],
                (float(self.cx[k]), float(self.cy[k]), float(self.cz[k])))

    def subset(self, idx) -> "Batch3":
        idx = np.asarray(idx, dtype=np.int64)
        sizes = self.sizes()[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(sizes, out=offs[1:])
        gather = np.repeat(self.offsets[idx] - offs[:-1], sizes) + np.arange(offs[-1], dtype=np.int64)
        return Batch3(offs, self.ax[gather], self.ay[gather], self.az[gather], self.b[gather], self.cx[idx],
                      self.cy[idx], self.cz[idx], self.kind[idx], self.box, self.name + "[subset]")

    def with_rows(self, ax=None, ay=None, az=None, b=None, box=None) -> "Batch3":
        pick = lambda new, old: old.copy() if new is None else np.ascontiguousarray(new, np.float32)
        return Batch3(self.offsets.copy(), pick(ax, self.ax), pick(ay, self.ay), pick(az, self.az), pick(b, self.b),
                      self.cx.copy(), self.cy.copy(), self.cz.copy(), self.kind.copy(),
                      self.box if box is None else box, self.name)

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.offsets, self.ax, self.ay, self.az, self.b, self.cx, self.cy, self.cz):
            h.update(np.ascontiguousarray(arr).tobytes())
        h.update(np.float64(self.box).tobytes())
        return h.hexdigest()


def concat3(batches, name="concat3") -> Batch3:
    boxes = {float(bt.box) for bt in batches}
    assert len(boxes) == 1, "batches with different boxes"
    sizes = np.concatenate([bt.sizes() for bt in batches])
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    cat = lambda f: np.concatenate([getattr(bt, f) for bt in batches])
    return Batch3(offs, cat("ax"), cat("ay"), cat("az"), cat("b"), cat("cx"), cat("cy"), cat("cz"), cat("kind"),
                  boxes.pop(), name)


def _unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def _insert(rng, n_rand, rand_rows, specials, n_spec):
    """Rows of B LPs: LP k gets its n_rand[k] random rows (LP-major, in order)
    with the first n_spec[k] rows of specials[k] inserted at uniform positions.
    Returns offsets and an (N, W) float64 array, W the width of a row."""
    B = n_rand.shape[0]
    K = specials.shape[1]
    sizes = n_rand + n_spec
    offsets = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    N = int(offsets[-1])
    rows = np.empty((N, rand_rows.shape[1]))
    pos = np.zeros((B, K), dtype=np.int64)
    for j in range(K):
        active = j < n_spec
        pj = np.minimum(np.floor(rng.random(B) * (n_rand + j + 1)).astype(np.int64), n_rand + j)
        pos[:, :j] += (pos[:, :j] >= pj[:, None]) & active[:, None]
        pos[:, j] = np.where(active, pj, 0)
    valid = np.arange(K)[None, :] < n_spec[:, None]
    gidx = (offsets[:-1, None] + pos)[valid]
    is_spec = np.zeros(N, dtype=bool)
    is_spec[gidx] = True
    rows[~is_spec] = rand_rows
    rows[gidx] = specials[valid]
    return offsets, rows


def uniform3_batch(num_lps: int, m: int, seed: int = 0, infeasible_frac=0.05, unbounded_frac=0.02,
                   box: float = 1.0e4, name=None) -> Batch3:
    """num_lps LPs with m random planes each: unit normals uniform on the
    sphere, offsets U[1, 2] (every LP contains the unit ball), a random unit
    objective.  The infeasible share also gets the pair a.x <= -3, -a.x <= -3
    at random positions; the unbounded share draws its normals from the
    hemisphere n.u >= 0 and its objective within 60 degrees of -u, so -u is a
    recession direction the objective climbs and the optimum is on the box."""
    rng = rng_for(31, num_lps, m, seed)
    kind = np.full(num_lps, KIND_BOXED, dtype=np.int64)
    perm = rng.permutation(num_lps)
    n_inf = int(round(infeasible_frac * num_lps))
    n_unb = int(round(unbounded_frac * num_lps))
    kind[perm[:n_inf]] = KIND_INFEASIBLE
    kind[perm[n_inf:n_inf + n_unb]] = KIND_UNBOUNDED

    n_rand = np.full(num_lps, m, dtype=np.int64)
    N = num_lps * m
    nrm = _unit_vectors(rng, N)
    off = 1.0 + rng.random(N)
    c = _unit_vectors(rng, num_lps)
    unb = kind == KIND_UNBOUNDED
    if unb.any():
        u = _unit_vectors(rng, num_lps)
        lp_of_row = np.repeat(np.arange(num_lps), m)
        flip = unb[lp_of_row] & (np.einsum("ij,ij->i", nrm, u[lp_of_row]) < 0.0)
        nrm[flip] = -nrm[flip]
        # objective: -u tilted by up to 60 degrees
        w = _unit_vectors(rng, num_lps)
        w -= np.einsum("ij,ij->i", w, u)[:, None] * u
        w /= np.maximum(np.linalg.norm(w, axis=1, keepdims=True), 1e-30)
        ang = rng.random(num_lps) * (np.pi / 3.0)
        cu = -np.cos(ang)[:, None] * u + np.sin(ang)[:, None] * w
        c[unb] = cu[unb]
    rand_rows = np.concatenate([nrm, off[:, None]], axis=1)
    specials = np.zeros((num_lps, 2, 4))
    n_spec = np.zeros(num_lps, dtype=np.int64)
    inf = kind == KIND_INFEASIBLE
    a = _unit_vectors(rng, num_lps).astype(np.float32).astype(np.float64)
    specials[:, 0, :3] = a
    specials[:, 0, 3] = -3.0
    specials[:, 1, :3] = -a
    specials[:, 1, 3] = -3.0
    n_spec[inf] = 2
    offsets, rows = _insert(rng, n_rand, rand_rows, specials, n_spec)
    f32 = lambda v: np.ascontiguousarray(v, dtype=np.float32)
    return Batch3(offsets, f32(rows[:, 0]), f32(rows[:, 1]), f32(rows[:, 2]), f32(rows[:, 3]), f32(c[:, 0]),
                  f32(c[:, 1]), f32(c[:, 2]), kind.astype(np.int8), float(box), name or f"uniform3_{num_lps}x{m}")


def tiny_integer_batch3(num_lps: int, m_max: int = 6, K: int = 3, seed: int = 0, m_min: int = 0,
                        zero_c_frac: float = 0.1, box: float = 64.0, boxed: bool = False) -> Batch3:
    """Small LPs with integer coefficients in [-K, K] (exact in fp32), so that
    degenerate cases (parallel and coincident planes, four planes through a
    point, zero normals, objectives normal to a face or zero) appear often.
    The box is a power of two beyond most vertices.  ``boxed`` also inserts
    the rows |x_k| <= K at random positions, which makes most LPs end inside
    the box."""
    if boxed:
        base = tiny_integer_batch3(num_lps, m_max, K, seed, m_min, zero_c_frac, box, boxed=False)
        rng = rng_for(34, num_lps, m_max, K, seed)
        sp = np.zeros((num_lps, 6, 4))
        for k in range(3):
            sp[:, 2 * k, k], sp[:, 2 * k + 1, k] = 1.0, -1.0
        sp[:, :, 3] = K
        rand_rows = np.stack([base.ax, base.ay, base.az, base.b], axis=1).astype(np.float64)
        offsets, rows = _insert(rng, base.sizes(), rand_rows, sp, np.full(num_lps, 6, dtype=np.int64))
        f32 = lambda v: np.ascontiguousarray(v, dtype=np.float32)
        return Batch3(offsets, f32(rows[:, 0]), f32(rows[:, 1]), f32(rows[:, 2]), f32(rows[:, 3]), base.cx, base.cy,
                      base.cz, base.kind, base.box, f"tiny_int3_boxed_{num_lps}")
    rng = rng_for(32, num_lps, m_max, K, seed)
    m = rng.integers(m_min, m_max + 1, num_lps)
    offsets = np.zeros(num_lps + 1, dtype=np.int64)
    np.cumsum(m, out=offsets[1:])
    N = int(offsets[-1])
    draw = lambda n: rng.integers(-K, K + 1, n).astype(np.float32)
    ax, ay, az, b = draw(N), draw(N), draw(N), draw(N)
    cx, cy, cz = draw(num_lps), draw(num_lps), draw(num_lps)
    z = rng.random(num_lps) < zero_c_frac
    cx[z] = cy[z] = cz[z] = 0.0
    return Batch3(offsets, ax, ay, az, b, cx, cy, cz, np.full(num_lps, KIND_OTHER, np.int8), float(box),
                  f"tiny_int3_{num_lps}")


def tiny_random_batch3(num_lps: int, m_max: int = 40, seed: int = 0, m_min: int = 0, box: float = 100.0) -> Batch3:
    """Small LPs with continuous coefficients: normals in random directions
    with length in [0.5, 2], offsets U[-0.5, 2], a random unit objective.  A
    good share ends up infeasible and some touch the box."""
    rng = rng_for(33, num_lps, m_max, seed)
    m = rng.integers(m_min, m_max + 1, num_lps)
    offsets = np.zeros(num_lps + 1, dtype=np.int64)
    np.cumsum(m, out=offsets[1:])
    N = int(offsets[-1])
    nrm = _unit_vectors(rng, N) * (0.5 + 1.5 * rng.random(N))[:, None]
    b = -0.5 + 2.5 * rng.random(N)
    c = _unit_vectors(rng, num_lps)
    f32 = lambda v: np.ascontiguousarray(v, dtype=np.float32)
    return Batch3(offsets, f32(nrm[:, 0]), f32(nrm[:, 1]), f32(nrm[:, 2]), f32(b), f32(c[:, 0]), f32(c[:, 1]),
                  f32(c[:, 2]), np.full(num_lps, KIND_OTHER, np.int8), float(box), f"tiny_rand3_{num_lps}")


CONFIGS3 = {
    # the 3D measurement workload: 65,536 LPs x 128 planes
    "uniform3": dict(num_lps=65536, m=128),
}


def make_config3(name: str, seed: int = 0, scale: float = 1.0) -> Batch3:
    cfg = dict(CONFIGS3[name])
    n = max(1, int(round(cfg.pop("num_lps") * scale)))
    return uniform3_batch(n, seed=seed, name=name, **cfg)
