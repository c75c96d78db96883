"""Seeded synthetic inputs for batched LPs in n dimensions (n = 2..5).

Like ``gen`` and ``gen3``, this module only draws random numbers and lays them
out; it holds none of the solver's arithmetic, so the oracle and the HIP path
both take their inputs from it.

Every LP is ``maximize c.x subject to a_i.x <= b_i`` over x in R^n (Eq. (1)-(2)
of the paper in n dimensions), inside the box ``|x_k| <= box`` (the bounding
rows of Sec. 2.1, given by the caller instead of stored as rows).  A batch is
stored CSR-offset SoA: ``offsets`` (int64, B+1), the normals ``a`` (float32,
shape (n, N): row i's k-th component is ``a[k, i]``), ``b`` (float32, N) and
the objectives ``c`` (float32, shape (n, B)).  The solver keeps the input
order, so the random row order Seidel's expected bound needs is drawn here.
The paper names higher dimensions as its next step (Sec. 6) and has no
workload for them; these recipes carry its 2D ones over exactly as the 3D
module does: random hyperplanes tangent to a sphere around the origin at
distance U[1, 2], a share made infeasible by an antiparallel pair with a gap,
and a share whose rows leave a recession direction open (reported as touching
the box).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

from .gen import KIND_BOXED, KIND_INFEASIBLE, KIND_OTHER, KIND_UNBOUNDED, rng_for
from .gen3 import _insert


@dataclasses.dataclass
class BatchN:
    offsets: np.ndarray
    a: np.ndarray      # (n, N) float32
    b: np.ndarray      # (N,) float32
    c: np.ndarray      # (n, B) float32
    kind: np.ndarray
    box: float
    name: str = ""

    @property
    def dim(self) -> int:
        return int(self.a.shape[0])

    @property
    def num_lps(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def num_constraints(self) -> int:
        return int(self.offsets[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def algorithmic_bytes(self) -> int:
        """One read of (a, b) per row plus, per LP, its offset, objective and
        the (x, status) it writes: 4 (n + 1) B * N + (8 + 8 n + 4) B * B."""
        n = self.dim
        return 4 * (n + 1) * self.num_constraints + (12 + 8 * n) * self.num_lps

    def lp(self, k: int):
        s, e = int(self.offsets[k]), int(self.offsets[k + 1])
        return self.a[:, s:e], self.b[s:e], self.c[:, k].astype(np.float64)

    def subset(self, idx) -> "BatchN":
        idx = np.asarray(idx, dtype=np.int64)
        sizes = self.sizes()[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(sizes, out=offs[1:])
        gather = np.repeat(self.offsets[idx] - offs[:-1], sizes) + np.arange(offs[-1], dtype=np.int64)
        return BatchN(offs, np.ascontiguousarray(self.a[:, gather]), self.b[gather],
                      np.ascontiguousarray(self.c[:, idx]), self.kind[idx], self.box, self.name + "[subset]")

    def with_rows(self, a=None, b=None, c=None, box=None) -> "BatchN":
        pick = lambda new, old: old.copy() if new is None else np.ascontiguousarray(new, np.float32)
        return BatchN(self.offsets.copy(), pick(a, self.a), pick(b, self.b), pick(c, self.c), self.kind.copy(),
                      self.box if box is None else box, self.name)

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.offsets, self.a, self.b, self.c):
            h.update(np.ascontiguousarray(arr).tobytes())
        h.update(np.float64(self.box).tobytes())
        return h.hexdigest()


def concat_n(batches, name="concat_n") -> BatchN:
    boxes = {float(bt.box) for bt in batches}
    dims = {bt.dim for bt in batches}
    assert len(boxes) == 1 and len(dims) == 1, "batches with different boxes or dimensions"
    sizes = np.concatenate([bt.sizes() for bt in batches])
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    return BatchN(offs, np.ascontiguousarray(np.concatenate([bt.a for bt in batches], axis=1)),
                  np.concatenate([bt.b for bt in batches]),
                  np.ascontiguousarray(np.concatenate([bt.c for bt in batches], axis=1)),
                  np.concatenate([bt.kind for bt in batches]), boxes.pop(), name)


def from_rows(rows, c, box, kind=None, name="rows") -> BatchN:
    """A batch from per-LP lists: rows[k] is an (m_k, n + 1) array of
    (a_1, ..., a_n, b), c[k] the objective."""
    n = len(c[0])
    sizes = np.array([len(r) for r in rows], dtype=np.int64)
    offs = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    flat = np.concatenate([np.asarray(r, np.float64).reshape(-1, n + 1) for r in rows]) if offs[-1] else \
        np.zeros((0, n + 1))
    B = len(rows)
    return BatchN(offs, np.ascontiguousarray(flat[:, :n].T, dtype=np.float32), np.ascontiguousarray(flat[:, n],
                  dtype=np.float32), np.ascontiguousarray(np.asarray(c, np.float64).T, dtype=np.float32),
                  np.full(B, KIND_OTHER, np.int8) if kind is None else np.asarray(kind, np.int8), float(box), name)


def _unit_vectors(rng, count, n):
    v = rng.standard_normal((count, n))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def uniform_n_batch(n: int, num_lps: int, m: int, seed: int = 0, infeasible_frac=0.05, unbounded_frac=0.02,
                    box: float = 1.0e4, name=None) -> BatchN:
    """num_lps LPs with m random hyperplanes each: unit normals uniform on the
    sphere S^(n-1), offsets U[1, 2] (every LP contains the unit ball), a
    random unit objective.  The infeasible share also gets the pair
    a.x <= -3, -a.x <= -3 at random positions; the unbounded share draws its
    normals from the hemisphere n.u >= 0 and its objective within 60 degrees
    of -u, so -u is a recession direction the objective climbs and the optimum
    is on the box."""
    rng = rng_for(41, n, num_lps, m, seed)
    kind = np.full(num_lps, KIND_BOXED, dtype=np.int64)
    perm = rng.permutation(num_lps)
    n_inf = int(round(infeasible_frac * num_lps))
    n_unb = int(round(unbounded_frac * num_lps))
    kind[perm[:n_inf]] = KIND_INFEASIBLE
    kind[perm[n_inf:n_inf + n_unb]] = KIND_UNBOUNDED

    N = num_lps * m
    nrm = _unit_vectors(rng, N, n)
    off = 1.0 + rng.random(N)
    c = _unit_vectors(rng, num_lps, n)
    unb = kind == KIND_UNBOUNDED
    if unb.any():
        u = _unit_vectors(rng, num_lps, n)
        lp_of_row = np.repeat(np.arange(num_lps), m)
        flip = unb[lp_of_row] & (np.einsum("ij,ij->i", nrm, u[lp_of_row]) < 0.0)
        nrm[flip] = -nrm[flip]
        w = _unit_vectors(rng, num_lps, n)
        w -= np.einsum("ij,ij->i", w, u)[:, None] * u
        w /= np.maximum(np.linalg.norm(w, axis=1, keepdims=True), 1e-30)
        ang = rng.random(num_lps) * (np.pi / 3.0)
        cu = -np.cos(ang)[:, None] * u + np.sin(ang)[:, None] * w
        c[unb] = cu[unb]
    rand_rows = np.concatenate([nrm, off[:, None]], axis=1)
    specials = np.zeros((num_lps, 2, n + 1))
    n_spec = np.zeros(num_lps, dtype=np.int64)
    inf = kind == KIND_INFEASIBLE
    a = _unit_vectors(rng, num_lps, n).astype(np.float32).astype(np.float64)
    specials[:, 0, :n] = a
    specials[:, 0, n] = -3.0
    specials[:, 1, :n] = -a
    specials[:, 1, n] = -3.0
    n_spec[inf] = 2
    offsets, rows = _insert(rng, np.full(num_lps, m, dtype=np.int64), rand_rows, specials, n_spec)
    return BatchN(offsets, np.ascontiguousarray(rows[:, :n].T, dtype=np.float32),
                  np.ascontiguousarray(rows[:, n], dtype=np.float32), np.ascontiguousarray(c.T, dtype=np.float32),
                  kind.astype(np.int8), float(box), name or f"uniform{n}_{num_lps}x{m}")


def tiny_integer_n_batch(n: int, num_lps: int, m_max: int = 6, K: int = 3, seed: int = 0, m_min: int = 0,
                         zero_c_frac: float = 0.1, box: float = 64.0, boxed: bool = False) -> BatchN:
    """Small LPs with integer coefficients in [-K, K] (exact in fp32), so that
    degenerate cases (parallel and coincident hyperplanes, more than n of them
    through a point, zero normals, objectives normal to a face or zero)
    appear often.  The box is a power of two beyond most vertices.  ``boxed``
    also inserts the rows |x_k| <= K at random positions, which makes most LPs
    end inside the box."""
    rng = rng_for(42, n, num_lps, m_max, K, seed)
    m = rng.integers(m_min, m_max + 1, num_lps)
    offsets = np.zeros(num_lps + 1, dtype=np.int64)
    np.cumsum(m, out=offsets[1:])
    N = int(offsets[-1])
    a = rng.integers(-K, K + 1, (n, N)).astype(np.float32)
    b = rng.integers(-K, K + 1, N).astype(np.float32)
    c = rng.integers(-K, K + 1, (n, num_lps)).astype(np.float32)
    c[:, rng.random(num_lps) < zero_c_frac] = 0.0
    bt = BatchN(offsets, a, b, c, np.full(num_lps, KIND_OTHER, np.int8), float(box), f"tiny_int{n}_{num_lps}")
    if not boxed:
        return bt
    rng2 = rng_for(43, n, num_lps, m_max, K, seed)
    sp = np.zeros((num_lps, 2 * n, n + 1))
    for k in range(n):
        sp[:, 2 * k, k], sp[:, 2 * k + 1, k] = 1.0, -1.0
    sp[:, :, n] = K
    rand_rows = np.concatenate([a.T, b[:, None]], axis=1).astype(np.float64)
    offsets, rows = _insert(rng2, m.astype(np.int64), rand_rows, sp, np.full(num_lps, 2 * n, dtype=np.int64))
    return BatchN(offsets, np.ascontiguousarray(rows[:, :n].T, dtype=np.float32),
                  np.ascontiguousarray(rows[:, n], dtype=np.float32), c, bt.kind, bt.box,
                  f"tiny_int{n}_boxed_{num_lps}")


def tiny_random_n_batch(n: int, num_lps: int, m_max: int = 20, seed: int = 0, m_min: int = 0,
                        box: float = 100.0) -> BatchN:
    """Small LPs with continuous coefficients: normals in random directions
    with length in [0.5, 2], offsets U[-0.5, 2], a random unit objective.  A
    good share ends up infeasible and some touch the box."""
    rng = rng_for(44, n, num_lps, m_max, seed)
    m = rng.integers(m_min, m_max + 1, num_lps)
    offsets = np.zeros(num_lps + 1, dtype=np.int64)
    np.cumsum(m, out=offsets[1:])
    N = int(offsets[-1])
    nrm = _unit_vectors(rng, N, n) * (0.5 + 1.5 * rng.random(N))[:, None]
    b = -0.5 + 2.5 * rng.random(N)
    c = _unit_vectors(rng, num_lps, n)
    return BatchN(offsets, np.ascontiguousarray(nrm.T, dtype=np.float32), b.astype(np.float32),
                  np.ascontiguousarray(c.T, dtype=np.float32), np.full(num_lps, KIND_OTHER, np.int8), float(box),
                  f"tiny_rand{n}_{num_lps}")


CONFIGSN = {
    # the 4D and 5D measurement workloads: 65,536 LPs of 128 and 64 hyperplanes
    "uniform4": dict(n=4, num_lps=65536, m=128),
    "uniform5": dict(n=5, num_lps=65536, m=64),
}


def make_config_n(name: str, seed: int = 0, scale: float = 1.0) -> BatchN:
    cfg = dict(CONFIGSN[name])
    k = max(1, int(round(cfg.pop("num_lps") * scale)))
    return uniform_n_batch(cfg.pop("n"), k, seed=seed, name=name, **cfg)
