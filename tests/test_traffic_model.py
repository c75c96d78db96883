"""The memory-row model of the binned kernel (paper_1902_04995_amd/traffic_model.py):
its counting rules on hand-made cases, and its totals on a small uneven sample."""
import numpy as np

from paper_1902_04995_amd import gen, traffic_model as tm


def test_rows_in_cache_and_chunk_are_not_reread():
    # 100 LPs of 40 rows (36 + the box): size class 6 runs 8 lanes per LP, whose share of the
    # wave's LDS cache is 56 rows, so no 1D LP reads memory and only the end-of-LP pass does
    bt = gen.uniform_batch(100, 36, seed=3)
    per = tm.model(bt)
    first, re, fin = np.sum(list(per.values()), axis=0)
    assert first == bt.num_constraints
    assert re == 0
    assert 0 < fin < first


def test_violation_order_matches_a_hand_case():
    # rows: x <= 4, y <= 3, x + y <= 5 with c = (1, 1): the start point violates all three
    ax = np.array([1, 0, 1], np.float32)
    ay = np.array([0, 1, 1], np.float32)
    b = np.array([4, 3, 5], np.float32)
    vs, dead = tm.violations(ax, ay, b, np.array([1.0, 1.0]))
    assert vs == [0, 1, 2] and not dead
    vs, dead = tm.violations(np.array([1, -1], np.float32), np.array([0, 0], np.float32),
                             np.array([1, -2], np.float32), np.array([1.0, 0.0]))
    assert dead  # x <= 1 and x >= 2


def test_uneven_sample_totals():
    per = tm.model(gen.uneven_batch(300, seed=7))
    first, re, fin = np.sum(list(per.values()), axis=0)
    assert 1.3 < (first + re) / first < 2.5
    assert fin > 0.3 * first
