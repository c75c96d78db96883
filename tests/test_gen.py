"""Input generators: shapes, seeds, mix counts and the shuffle (CPU only)."""
import math

import numpy as np

from paper_1902_04995_amd import gen


def test_uniform_shapes_and_mix():
    bt = gen.uniform_batch(2000, 256, seed=0)
    sizes = bt.sizes()
    kind = bt.kind
    assert bt.offsets[0] == 0 and bt.offsets.dtype == np.int64
    assert bt.ax.dtype == np.float32 and bt.cx.dtype == np.float32
    assert np.all(sizes[kind == gen.KIND_BOXED] == 260)
    assert np.all(sizes[kind == gen.KIND_INFEASIBLE] == 262)
    assert np.all(sizes[kind == gen.KIND_UNBOUNDED] == 256)
    assert (kind == gen.KIND_INFEASIBLE).sum() == 100 and (kind == gen.KIND_UNBOUNDED).sum() == 40
    assert np.allclose(np.hypot(bt.cx, bt.cy), 1.0, atol=1e-6)


def test_seed_determinism():
    a = gen.uniform_batch(300, 64, seed=5)
    b = gen.uniform_batch(300, 64, seed=5)
    c = gen.uniform_batch(300, 64, seed=6)
    assert a.digest() == b.digest() != c.digest()


def test_special_rows_are_uniformly_placed():
    """The box rows land at uniform positions: their mean relative position is 1/2."""
    bt = gen.uniform_batch(4000, 60, seed=1, infeasible_frac=0.0, unbounded_frac=0.0)
    is_box = bt.b == np.float32(1e6)
    pos = np.flatnonzero(is_box) - np.repeat(bt.offsets[:-1], 4)
    rel = pos / 63.0
    assert abs(rel.mean() - 0.5) < 0.01
    assert np.all(np.bincount(np.repeat(np.arange(4000), 4), minlength=4000) == 4)
    assert is_box.reshape(-1).sum() == 16000


def test_uneven_log_uniform():
    bt = gen.uneven_batch(4000, 8, 8192, seed=2, infeasible_frac=0.0, unbounded_frac=0.0)
    m = bt.sizes() - 4
    assert m.min() >= 8 and m.max() <= 8192
    lm = np.log(m)
    assert abs(np.median(lm) - 0.5 * (math.log(8) + math.log(8193))) < 0.1


def test_crowd_shape():
    bt = gen.crowd_batch(4096, seed=3)
    k = bt.sizes() - 16
    assert k.min() >= 8 and k.max() <= 64
    assert np.allclose(np.hypot(bt.ax, bt.ay), 1.0, atol=1e-6)
    assert (bt.b < 0).any()  # some agents overlap a neighbour


def test_subset_and_concat_roundtrip():
    bt = gen.uneven_batch(100, 8, 64, seed=4)
    idx = np.array([5, 0, 99, 17])
    sub = bt.subset(idx)
    for j, k in enumerate(idx):
        for u, v in zip(sub.lp(j), bt.lp(int(k))):
            assert np.array_equal(np.asarray(u), np.asarray(v))
    cat = gen.concat([sub, sub])
    assert cat.num_lps == 8 and cat.num_constraints == 2 * sub.num_constraints
