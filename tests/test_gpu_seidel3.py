"""GPU parity of the 3D solver (rgb_solve3_batch) against the 3D oracle.

Bar (per LP): status bit-exact; for OPTIMAL and UNBOUNDED (the optimum on the
box) ||x - x_oracle||_inf <= 1e-4 * max(1, |x_oracle|) per component (an FP64
solve rounded to FP32 against FP64 vertex enumeration).  Every lane width must
give bit-identical results (the bound reductions are exact min/max with a
smallest-index tie-break).
"""
import os
import sys

import numpy as np
import pytest

import lpcheck
from lpcheck import INFEASIBLE, INVALID, OPTIMAL, UNBOUNDED
from paper_1902_04995_amd import gen3

pytestmark = pytest.mark.gpu
X_RTOL = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rgb():
    import torch
    assert torch.cuda.is_available()
    import paper_1902_04995_amd as rgb
    rgb.lib()
    return rgb


def _run(rgb, bt, g=0):
    import torch
    dev = rgb.DeviceBatch3(bt, "cuda:0")
    x, y, z, st = dev.solve(lanes_per_lp=g)
    torch.cuda.synchronize()
    return st.cpu().numpy(), np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1)


def _mismatches(ref, st, x, idx=None):
    rs, rx = ref["status"], ref["x"]
    if idx is not None:
        rs, rx = rs[idx], rx[idx]
    bad_s = np.flatnonzero(st != rs)
    has_x = (rs == OPTIMAL) | (rs == UNBOUNDED)
    err = np.abs(x.astype(np.float64) - rx) > X_RTOL * np.maximum(1.0, np.abs(rx))
    bad_x = np.flatnonzero(has_x & (st == rs) & err.any(axis=1))
    return bad_s, bad_x


def _check(bt, ref, st, x, label):
    bs, bx = _mismatches(ref, st, x)
    msg = f"{label}: {len(bs)} status / {len(bx)} x mismatches of {bt.num_lps}"
    for k in list(bs[:5]) + list(bx[:5]):
        msg += f"\n  lp {k} m={bt.sizes()[k]} got st={st[k]} x={x[k]} ref st={ref['status'][k]} x={ref['x'][k]}"
    assert len(bs) + len(bx) == 0, msg


BATCHES = {
    "int_k2": lambda: gen3.tiny_integer_batch3(3000, m_max=8, K=2, seed=21),
    "int_k3_boxed": lambda: gen3.tiny_integer_batch3(3000, m_max=10, K=3, seed=22, boxed=True),
    "int_k1_boxed": lambda: gen3.tiny_integer_batch3(2000, m_max=12, K=1, seed=23, boxed=True),
    "random": lambda: gen3.tiny_random_batch3(3000, m_max=40, seed=24),
    "uniform3_small": lambda: gen3.uniform3_batch(2000, 64, seed=25),
}


@pytest.mark.parametrize("name", list(BATCHES))
def test_seidel3_matches_oracle(rgb, oracle_lib, name):
    bt = BATCHES[name]()
    ref = oracle_lib.solve3(bt)
    _say(f"[seidel3] {name}: {bt.num_lps} LPs, {bt.num_constraints} rows, status mix "
         f"{np.bincount(ref['status'], minlength=4).tolist()}")
    st, x = _run(rgb, bt)
    _check(bt, ref, st, x, name)


@pytest.mark.parametrize("g", [4, 8, 16, 32, 64])
def test_seidel3_lane_widths_bit_identical(rgb, oracle_lib, g):
    bt = gen3.concat3([gen3.uniform3_batch(700, 100, seed=26), gen3.uniform3_batch(300, 7, seed=27)])
    st0, x0 = _run(rgb, bt, 16)
    st, x = _run(rgb, bt, g)
    assert np.array_equal(st, st0)
    assert np.array_equal(x.view(np.int32), x0.view(np.int32))
    if g == 4:
        _check(bt, oracle_lib.solve3(bt), st, x, "uniform3 mix")


def test_seidel3_hand_solved_golden(rgb):
    lps = lpcheck.parse_golden3(os.path.join(lpcheck.GOLDEN, "lp3_hand.txt"))
    for lp, bt in zip(lps, lpcheck.golden3_batch(lps)):
        st, x = _run(rgb, bt)
        want, xyz = lp["expect"]
        assert st[0] == want, lp["name"]
        if xyz is None:
            assert np.isnan(x[0]).all(), lp["name"]
        else:
            np.testing.assert_allclose(x[0], xyz, rtol=1e-6, atol=1e-6, err_msg=lp["name"])


def test_seidel3_edges(rgb, oracle_lib):
    import torch
    # empty batch: nothing enqueued, no error
    z64 = torch.zeros(1, dtype=torch.int64, device="cuda")
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    out = rgb.solve3_batch(z64, e, e, e, e, e, e, e, 10.0)
    assert out[3].numel() == 0
    # empty LPs, NaN rows, NaN objective, bad offsets
    bt = gen3.tiny_random_batch3(40, m_max=12, m_min=0, seed=28)
    sizes = bt.sizes()
    ax = bt.ax.copy()
    b = bt.b.copy()
    cz = bt.cz.copy()
    k1 = int(np.flatnonzero(sizes >= 3)[0])
    k2 = int(np.flatnonzero(sizes >= 3)[1])
    ax[bt.offsets[k1] + 2] = np.nan
    b[bt.offsets[k2] + sizes[k2] - 1] = -np.inf
    cz[5] = np.inf
    bad = gen3.Batch3(bt.offsets, ax, bt.ay, bt.az, b, bt.cx, bt.cy, cz, bt.kind, bt.box)
    ref = oracle_lib.solve3(bad)
    st, x = _run(rgb, bad)
    assert st[k1] == INVALID and st[k2] == INVALID and st[5] == INVALID
    _check(bad, ref, st, x, "edges")
    assert (sizes == 0).any() and (st[sizes == 0] == UNBOUNDED).all()
    # offsets out of range, decreasing: INVALID, and nothing read out of range
    dev = rgb.DeviceBatch3(bt, "cuda:0")
    offs = dev.offsets.clone()
    offs[3] = bt.num_constraints + 100
    offs[7] = -5
    x_, y_, z_, s_ = rgb.solve3_batch(offs, dev.ax, dev.ay, dev.az, dev.b, dev.cx, dev.cy, dev.cz, bt.box)
    torch.cuda.synchronize()
    s_ = s_.cpu().numpy()
    assert s_[2] == INVALID and s_[3] == INVALID and s_[6] == INVALID and s_[7] == INVALID
    # argument errors are synchronous and enqueue nothing
    for box in (0.0, -1.0, float("inf"), float("nan"), 1e39):
        with pytest.raises(rgb.RgbError):
            rgb.solve3_batch(dev.offsets, dev.ax, dev.ay, dev.az, dev.b, dev.cx, dev.cy, dev.cz, box)
    with pytest.raises(rgb.RgbError):
        dev.solve(lanes_per_lp=12)


def test_seidel3_full_size_sampled(rgb, oracle_lib):
    """The measurement workload (65,536 LPs x 128 planes) in one launch at the
    default width; 384 sampled LPs against the oracle, and the status mix the
    generator plants (5% infeasible, 2% on the box)."""
    import torch
    bt = gen3.make_config3("uniform3", seed=0)
    st, x = _run(rgb, bt)
    rng = np.random.default_rng(29)
    idx = np.sort(rng.choice(bt.num_lps, 384, replace=False))
    sub = bt.subset(idx)
    ref = oracle_lib.solve3(sub)
    bs, bx = _mismatches(ref, st[idx], x[idx])
    assert len(bs) + len(bx) == 0, (bs[:5], bx[:5])
    counts = np.bincount(st, minlength=4)
    _say(f"[seidel3] full size status mix {counts.tolist()}")
    assert counts[INFEASIBLE] == int(round(0.05 * bt.num_lps))
    assert counts[UNBOUNDED] == int(round(0.02 * bt.num_lps))
    assert counts[INVALID] == 0
    # a second launch gives the same bits
    st2, x2 = _run(rgb, bt)
    assert np.array_equal(st2, st) and np.array_equal(x2.view(np.int32), x.view(np.int32))
    torch.cuda.empty_cache()


def test_seidel3_one_huge_lp(rgb):
    """One LP of 200,000 planes tangent to the unit sphere (Fibonacci lattice,
    random row order) among small ones: checked by properties that hold at
    any size -- every row satisfied, a KKT certificate on the tight rows, and
    the circumscribed-sphere band |c| <= c.x <= |c| / cos(r) (r the lattice's
    covering radius, bounded generously)."""
    import math
    n = 200_000
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = math.pi * (1 + 5 ** 0.5) * i
    nrm = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    perm = np.random.default_rng(30).permutation(n)
    nrm = nrm[perm].astype(np.float32)
    c = np.array([0.3, -0.5, 0.8], np.float32)
    big = gen3.Batch3(np.array([0, n], np.int64), nrm[:, 0].copy(), nrm[:, 1].copy(), nrm[:, 2].copy(),
                      np.ones(n, np.float32), c[:1], c[1:2], c[2:], np.zeros(1, np.int8), 1e4)
    bt = gen3.concat3([gen3.uniform3_batch(3000, 20, seed=31), big, gen3.uniform3_batch(2000, 9, seed=32)])
    k = 3000
    for g in (16, 64):
        st, x = _run(rgb, bt, g)
        assert st[k] == OPTIMAL, (g, st[k])
        xk = x[k].astype(np.float64)
        A = nrm.astype(np.float64)
        b = np.ones(n)
        viol, resid = lpcheck.kkt_residual3(A, b, c.astype(np.float64), xk, tight_tol=2e-6)
        assert viol <= 2e-6 and resid <= 1e-3, (g, viol, resid)
        cn = float(np.linalg.norm(c.astype(np.float64)))
        cosr = math.cos(2.0 * math.sqrt(math.pi / n))
        val = float(c.astype(np.float64) @ xk)
        assert cn * (1 - 1e-6) <= val <= cn / cosr * (1 + 1e-6), (val, cn)


def test_seidel3_lp_over_row_limit(rgb, oracle_lib):
    """One LP of 2^30 + 1 planes (over the per-LP limit, ~17 GB of real rows in
    device memory) is INVALID and never read; the 100-plane LP after it is
    still solved, at two lane widths."""
    import torch
    big = (1 << 30) + 1
    n = big + 100
    free, _ = torch.cuda.mem_get_info()
    if free < 16 * n + (2 << 30):
        pytest.skip(f"needs {16 * n / 2**30:.1f} GiB of free device memory, {free / 2**30:.1f} free")
    small = gen3.uniform3_batch(1, 100, seed=33, infeasible_frac=0.0, unbounded_frac=0.0)
    _say(f"[seidel3] case=over_limit rows={n}")
    cols = []
    for a in (small.ax, small.ay, small.az, small.b):
        t = torch.zeros(n, dtype=torch.float32, device="cuda")
        t[big:] = torch.from_numpy(a).cuda()
        cols.append(t)
    offs = torch.tensor([0, big, n], dtype=torch.int64, device="cuda")
    c = [torch.from_numpy(np.concatenate([[0.3], v]).astype(np.float32)).cuda() for v in (small.cx, small.cy, small.cz)]
    ref = oracle_lib.solve3(small)
    for g in (16, 64):
        x, y, z, st = rgb.solve3_batch(offs, *cols, *c, small.box, lanes_per_lp=g)
        torch.cuda.synchronize()
        st = st.cpu().numpy()
        xyz = np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1)
        assert st[0] == INVALID and np.isnan(xyz[0]).all(), g
        bs, bx = _mismatches(ref, st[1:], xyz[1:])
        assert len(bs) + len(bx) == 0, (g, st[1], xyz[1], ref["status"], ref["x"])
    del cols
    torch.cuda.empty_cache()
