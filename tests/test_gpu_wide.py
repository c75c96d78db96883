"""GPU: a batch of more than 2^30 rows, which takes the kernels' 64-bit row
indexing (every other test stays below it).  The batch is generated in device
memory (~13 GB); all kernel families must agree bit for bit, and a sample of
LPs is checked against the oracle.  The same rows then hold one LP of more
than 2^30 rows, which every family must report INVALID without reading it."""
import sys

import numpy as np
import pytest

import lpcheck
from paper_1902_04995_amd import gen

pytestmark = pytest.mark.gpu

M = 256
B = (1 << 22) + 1  # B * M = 2^30 + 256 rows


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_more_than_2_30_rows(oracle_lib):
    import torch
    assert torch.cuda.is_available()
    import paper_1902_04995_amd as rgb
    free, _ = torch.cuda.mem_get_info()
    need = 3 * 4 * B * M + 64 * B
    if free < need + (2 << 30):
        pytest.skip(f"needs {need / 2**30:.1f} GiB of free device memory, {free / 2**30:.1f} free")
    _say(f"[gpu] case=wide lps={B} rows={B * M}")
    offsets, ax, ay, b, cx, cy = gen.device_disk_batch(B, M, seed=30)
    assert ax.numel() > (1 << 30)
    torch.cuda.synchronize()
    results = {}
    for variant, g in (("plain", 0), ("batched", 32), ("persistent", 0), ("binned", 0), ("pooled", 8)):
        _say(f"[gpu] case=wide variant={variant} G={g}")
        x, y, st = rgb.solve_batch(offsets, ax, ay, b, cx, cy, variant=variant, lanes_per_lp=g)
        torch.cuda.synchronize()
        results[variant] = (st.cpu().numpy(), x.cpu().numpy(), y.cpu().numpy())
        del x, y, st
    base = results["plain"]
    for variant, got in results.items():
        for a, r, name in zip(got, base, ("status", "x", "y")):
            assert np.array_equal(a, r, equal_nan=True), f"{variant} differs from plain in {name}"
    # sample, including the LPs whose rows sit past row 2^30
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(B, 1500, replace=False), np.arange(B - 40, B)]))
    sub = gen.host_subset(offsets, ax, ay, b, cx, cy, idx)
    ref = oracle_lib.solve(sub)
    st, x, y = (a[idx] for a in base)
    bs, bx = lpcheck.compare(st, x.astype(np.float64), y.astype(np.float64), ref["status"], ref["x"], ref["y"])
    assert len(bs) == 0 and len(bx) == 0, (len(bs), len(bx))
    assert np.all(st == 0)  # every LP contains the unit disk and has 256 spread normals
    # the same rows as LPs of 4,096 rows (the last one the 256 rows past 2^30): the size
    # classes above 2,048 rows, whose kernels record where their 1D-LP bounds were reached,
    # with 64-bit row indexing
    B4 = (B * M + 4095) // 4096
    offs4 = torch.clamp(torch.arange(B4 + 1, device="cuda", dtype=torch.int64) * 4096, max=B * M)
    res4 = {}
    for variant, g in (("plain", 0), ("batched", 64), ("binned", 0)):
        _say(f"[gpu] case=wide_4096 variant={variant} G={g} lps={B4}")
        x, y, st = rgb.solve_batch(offs4, ax, ay, b, cx[:B4], cy[:B4], variant=variant, lanes_per_lp=g)
        torch.cuda.synchronize()
        res4[variant] = (st.cpu().numpy(), x.cpu().numpy(), y.cpu().numpy())
        del x, y, st
    for variant, got in res4.items():
        for a, r, name in zip(got, res4["plain"], ("status", "x", "y")):
            assert np.array_equal(a, r, equal_nan=True), f"4096-row LPs: {variant} differs from plain in {name}"
    idx4 = np.unique(np.concatenate([rng.choice(B4, 300, replace=False), np.arange(B4 - 5, B4)]))
    ref4 = oracle_lib.solve(gen.host_subset(offs4, ax, ay, b, cx[:B4], cy[:B4], idx4))
    st, x, y = (a[idx4] for a in res4["plain"])
    bs, bx = lpcheck.compare(st, x.astype(np.float64), y.astype(np.float64), ref4["status"], ref4["x"], ref4["y"])
    assert len(bs) == 0 and len(bx) == 0, (len(bs), len(bx))
    assert np.all(st == 0)
    del offs4, res4
    # one LP of 2^30 + 1 rows (over the per-LP limit): INVALID in every family,
    # its rows never read; the LP after it (the next 100 rows) still solved
    big = (1 << 30) + 1
    offs2 = torch.tensor([0, big, big + 100], dtype=torch.int64, device="cuda")
    sub2 = gen.host_subset(offs2, ax, ay, b, cx[:2], cy[:2], np.array([1]))
    ref2 = oracle_lib.solve(sub2)
    for variant, g in (("plain", 0), ("batched", 32), ("persistent", 0), ("binned", 0), ("pooled", 8)):
        _say(f"[gpu] case=over_limit variant={variant} G={g}")
        x, y, st = rgb.solve_batch(offs2, ax, ay, b, cx[:2], cy[:2], variant=variant, lanes_per_lp=g)
        torch.cuda.synchronize()
        st, x, y = st.cpu().numpy(), x.cpu().numpy(), y.cpu().numpy()
        assert st[0] == lpcheck.INVALID and np.isnan(x[0]) and np.isnan(y[0]), variant
        bs, bx = lpcheck.compare(st[1:], x[1:].astype(np.float64), y[1:].astype(np.float64),
                                 ref2["status"], ref2["x"], ref2["y"])
        assert len(bs) == 0 and len(bx) == 0, variant
