"""GPU: the host-to-host path (rgb_solve_batch_host).  Whatever the chunking
and whether the host buffers are pinned or pageable, results must equal the
device-resident solve of the same batch bit for bit (and so the oracle)."""
import sys

import numpy as np
import pytest

import lpcheck
from paper_1902_04995_amd import gen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _device_solve(rgb, bt, variant):
    import torch
    x, y, st = rgb.DeviceBatch(bt, "cuda:0").solve(variant=variant)
    torch.cuda.synchronize()
    return x.cpu().numpy(), y.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("variant", ["persistent", "batched", "pooled"])
def test_host_path_matches_device(oracle_lib, variant):
    import torch
    import paper_1902_04995_amd as rgb
    bt = gen.concat([gen.uneven_batch(1500, 8, 1200, seed=21), gen.tiny_random_batch(400, m_max=50, seed=22),
                     gen.uniform_batch(3, 3000, seed=23)])
    ref = _device_solve(rgb, bt, variant)
    o = oracle_lib.solve(bt)
    bs, bx = lpcheck.compare(ref[2], ref[0], ref[1], o["status"], o["x"], o["y"])
    assert len(bs) == 0 and len(bx) == 0
    for chunk_rows in (20000, 100, 0):
        _say(f"[gpu] host path {variant} pageable chunk_rows={chunk_rows}")
        x, y, st, ms = rgb.solve_batch_host(bt.offsets, bt.ax, bt.ay, bt.b, bt.cx, bt.cy, variant=variant,
                                            chunk_rows=chunk_rows)
        assert ms > 0
        for a, r in zip((x, y, st), ref):
            assert np.array_equal(a, r, equal_nan=True), (variant, chunk_rows)
    _say(f"[gpu] host path {variant} pinned")
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    args = [pin(bt.offsets)] + [pin(a) for a in (bt.ax, bt.ay, bt.b, bt.cx, bt.cy)]
    out = (torch.empty(bt.num_lps, dtype=torch.float32).pin_memory(),
           torch.empty(bt.num_lps, dtype=torch.float32).pin_memory(),
           torch.empty(bt.num_lps, dtype=torch.int32).pin_memory())
    x, y, st, _ = rgb.solve_batch_host(*args, variant=variant, chunk_rows=50000, out=out)
    for a, r in zip((x.numpy(), y.numpy(), st.numpy()), ref):
        assert np.array_equal(a, r, equal_nan=True), variant


def test_host_path_offsets_past_row_zero_and_errors():
    import paper_1902_04995_amd as rgb
    bt = gen.uniform_batch(200, 64, seed=24)
    ref = _device_solve(rgb, bt, "batched")
    # the same LPs with 7 unused rows in front: offsets start at row 7
    pad = lambda a: np.concatenate([np.full(7, 9.0, np.float32), a])
    offs = bt.offsets + 7
    x, y, st, _ = rgb.solve_batch_host(offs, pad(bt.ax), pad(bt.ay), pad(bt.b), bt.cx, bt.cy, variant="batched",
                                       chunk_rows=3000)
    for a, r in zip((x, y, st), ref):
        assert np.array_equal(a, r, equal_nan=True)
    bad = bt.offsets.copy()
    bad[5] = bad[4] - 1
    with pytest.raises(rgb.RgbError):
        rgb.solve_batch_host(bad, bt.ax, bt.ay, bt.b, bt.cx, bt.cy)
    with pytest.raises(rgb.RgbError):  # offsets past the rows
        rgb.solve_batch_host(bt.offsets + 1, bt.ax, bt.ay, bt.b, bt.cx, bt.cy)
