"""CPU: pins of the crowd-step reference (oracle/crowd.py)."""
import math

import numpy as np
import pytest

from oracle import crowd as cr


def test_splitmix64_published_value_and_two_forms():
    # the first output of SplitMix64 seeded with 0, as published with the generator
    assert cr.splitmix64_stream(0, 1)[0] == 16294208416658607535
    for seed in (0, 1, 12345, 2**63 + 7):
        seq = cr.splitmix64_stream(seed, 300)
        nth = cr.splitmix64_nth(seed, np.arange(1, 301, dtype=np.uint64))
        assert [int(v) for v in nth] == seq


def _crowd(n, seed, side=None):
    rng = np.random.default_rng(seed)
    side = side or math.sqrt(n)
    px = (rng.random(n) * side).astype(np.float32)
    py = (rng.random(n) * side).astype(np.float32)
    k = rng.integers(8, 65, n).astype(np.int32)
    k = np.minimum(k, n - 1)
    return px, py, k


@pytest.mark.parametrize("seed", [1, 2])
def test_knn_matches_brute_force(seed):
    px, py, k = _crowd(300, seed)
    px[5], py[5] = px[7], py[7]  # a coincident pair (distance 0)
    px[11], py[11] = px[3] + np.float32(1.0), py[3]  # equal distances from agent 3 ...
    px[12], py[12] = px[3] - np.float32(1.0), py[3]  # ... broken by index
    assert cr.knn(px, py, k) == cr.knn_brute(px, py, k)


def test_rows_are_the_neighbour_and_disc_half_planes():
    px, py, k = _crowd(200, 3)
    nbrs = cr.knn(px, py, k)
    offs, ax, ay, b = cr.build_rows(px, py, k, nbrs, 0.3, 1.0, 16, seed=9, step=4)
    assert np.array_equal(np.diff(offs), k.astype(np.int64) + 16)
    from scipy.optimize import linear_sum_assignment
    for i in range(200):
        s, e = offs[i], offs[i + 1]
        got = np.stack([ax[s:e], ay[s:e], b[s:e]], axis=1).astype(np.float64)
        want = []
        for j in nbrs[i]:
            d = math.hypot(float(px[j]) - float(px[i]), float(py[j]) - float(py[i]))
            want.append(((float(px[j]) - float(px[i])) / d, (float(py[j]) - float(py[i])) / d, 0.5 * (d - 0.3)))
        for q in range(16):
            want.append((math.cos(2 * math.pi * q / 16), math.sin(2 * math.pi * q / 16), 1.0))
        want = np.array(want)
        cost = np.abs(got[:, None, :] - want[None, :, :]).max(axis=2)
        r, c = linear_sum_assignment(cost)  # the rows are the wanted ones, in some order
        assert cost[r, c].max() < 1e-5


def test_row_order_depends_on_seed_step_and_agent_only():
    px, py, k = _crowd(50, 4)
    nbrs = cr.knn(px, py, k)
    a = cr.build_rows(px, py, k, nbrs, 0.3, 1.0, 16, seed=1, step=0)
    b = cr.build_rows(px, py, k, nbrs, 0.3, 1.0, 16, seed=1, step=0)
    c = cr.build_rows(px, py, k, nbrs, 0.3, 1.0, 16, seed=1, step=1)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[1], c[1])
    assert np.array_equal(np.sort(a[1]), np.sort(c[1]))  # the same rows, another order
