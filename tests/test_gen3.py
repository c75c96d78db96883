"""CPU checks of the 3D input generators: layout, determinism, and the recipe
the parity tests and the measurement rely on."""
import numpy as np

from paper_1902_04995_amd import gen, gen3


def test_uniform3_layout_and_recipe():
    bt = gen3.uniform3_batch(2000, 32, seed=3)
    assert bt.offsets[0] == 0 and np.all(np.diff(bt.offsets) >= 0) and bt.offsets[-1] == bt.ax.size
    for a in (bt.ax, bt.ay, bt.az, bt.b, bt.cx, bt.cy, bt.cz):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    sizes = bt.sizes()
    inf = bt.kind == gen.KIND_INFEASIBLE
    unb = bt.kind == gen.KIND_UNBOUNDED
    assert inf.sum() == 100 and unb.sum() == 40
    assert np.all(sizes[inf] == 34) and np.all(sizes[~inf] == 32)
    # every random row keeps the unit ball inside (|n| = 1, b in [1, 2]); the
    # infeasible pair is the only exception
    nrm = np.sqrt(bt.ax.astype(np.float64) ** 2 + bt.ay ** 2 + bt.az ** 2)
    pair = np.isclose(bt.b, -3.0)
    assert pair.sum() == 2 * inf.sum()
    assert np.allclose(nrm[~pair], 1.0, atol=1e-6) and np.all((bt.b[~pair] >= 1.0) & (bt.b[~pair] <= 2.0))
    # the unbounded share has a recession direction the objective climbs
    # (some r with A r <= 0 and c.r > 0); the bounded share has none
    from scipy.optimize import linprog
    for k in list(np.flatnonzero(unb)[:8]) + list(np.flatnonzero(~unb & ~inf)[:8]):
        ax, ay, az, b, c = bt.lp(k)
        A = np.stack([ax, ay, az], 1).astype(np.float64)
        r = linprog(-np.array(c, np.float64), A_ub=A, b_ub=np.zeros(len(b)), bounds=[(-1, 1)] * 3, method="highs")
        assert r.status == 0
        assert (-r.fun > 1e-6) == bool(unb[k]), (k, -r.fun)
    assert bt.algorithmic_bytes() == 16 * bt.num_constraints + 36 * bt.num_lps


def test_generators3_deterministic_and_subset():
    a = gen3.make_config3("uniform3", seed=4, scale=500 / 65536)
    b = gen3.make_config3("uniform3", seed=4, scale=500 / 65536)
    assert a.digest() == b.digest()
    assert gen3.make_config3("uniform3", seed=5, scale=500 / 65536).digest() != a.digest()
    idx = np.array([7, 3, 499, 0])
    sub = a.subset(idx)
    for j, k in enumerate(idx):
        for x, y in zip(sub.lp(j)[:4], a.lp(k)[:4]):
            assert np.array_equal(x, y)
        assert sub.lp(j)[4] == a.lp(k)[4]


def test_tiny_integer3_boxed_inserts_box_rows():
    base = gen3.tiny_integer_batch3(300, m_max=6, K=2, seed=6)
    boxed = gen3.tiny_integer_batch3(300, m_max=6, K=2, seed=6, boxed=True)
    assert np.array_equal(boxed.sizes(), base.sizes() + 6)
    for k in range(0, 300, 37):
        ax, ay, az, b, c = boxed.lp(k)
        rows = {(float(p), float(q), float(r), float(s)) for p, q, r, s in zip(ax, ay, az, b)}
        for e in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            assert (*map(float, e), 2.0) in rows
        assert c == boxed.lp(k)[4] == base.lp(k)[4]
    assert np.all(np.abs(base.ax) <= 2) and np.all(base.ax == np.round(base.ax))
