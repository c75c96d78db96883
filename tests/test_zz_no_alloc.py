"""rgb_solve_batch_noalloc, the entry point that allocates nothing, against
rgb_solve_batch on the same batches (through the C ABI): two calls in a row on
one device, the second with a smaller batch, for both families that keep
their binning state in the library's static workspace, and the size limit."""
import numpy as np
import pytest

from paper_1902_04995_amd import gen

pytestmark = pytest.mark.gpu


def _host(out):
    return tuple(t.cpu().numpy() for t in out)


def _same(a, b, what):
    xa, ya, sa = a
    xb, yb, sb = b
    assert np.array_equal(sa, sb), (what, np.flatnonzero(sa != sb)[:10])
    # the same kernels run on the same rows: bit-identical, which is within
    # the 1e-4 * max(1, |x|) bar of the parity tests
    assert np.array_equal(xa, xb, equal_nan=True), what
    assert np.array_equal(ya, yb, equal_nan=True), what


@pytest.mark.parametrize("variant", ["binned", "persistent"])
def test_noalloc_matches_solve_batch_twice(variant):
    import torch

    import paper_1902_04995_amd as rgb
    big = gen.concat([gen.uneven_batch(6000, m_lo=8, m_hi=4096, seed=31),
                      gen.tiny_random_batch(800, m_max=40, seed=32)])
    small = gen.uniform_batch(1500, 96, seed=33)
    assert small.num_lps < big.num_lps
    for bt in (big, small):
        dev = rgb.DeviceBatch(bt, "cuda:0")
        ref = dev.solve(variant=variant)
        torch.cuda.synchronize()
        ref = _host(ref)
        out = (torch.full((bt.num_lps,), 7.0, dtype=torch.float32, device="cuda"),
               torch.full((bt.num_lps,), 7.0, dtype=torch.float32, device="cuda"),
               torch.full((bt.num_lps,), 9, dtype=torch.int32, device="cuda"))
        rgb.solve_batch_noalloc(dev.offsets, dev.ax, dev.ay, dev.b, dev.cx, dev.cy, out=out, variant=variant)
        torch.cuda.synchronize()
        got = _host(out)
        _same(got, ref, (variant, bt.name, bt.num_lps))
        assert np.all(got[2] <= 3), "a status outside rgb_status_t"


def test_noalloc_rejects_batches_over_the_limit():
    import torch

    import paper_1902_04995_amd as rgb
    n = (1 << 20) + 1
    offsets = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    row = torch.zeros(1, dtype=torch.float32, device="cuda")
    c = torch.zeros(n, dtype=torch.float32, device="cuda")
    out = (torch.empty(n, dtype=torch.float32, device="cuda"), torch.empty(n, dtype=torch.float32, device="cuda"),
           torch.full((n,), 9, dtype=torch.int32, device="cuda"))
    with pytest.raises(rgb.RgbError, match=r"\(-5\)"):
        rgb.solve_batch_noalloc(offsets, row[:0], row[:0], row[:0], c, c, out=out, variant="binned")
    torch.cuda.synchronize()
    assert bool((out[2] == 9).all()), "nothing may be written when the batch is refused"


@pytest.mark.parametrize("variant", ["binned", "persistent"])
def test_noalloc_under_graph_capture(variant):
    """The use the entry point exists for: a solve captured into a HIP graph
    (where the context's workspace could not be grown) and replayed several
    times, with eager work and synchronisations between the replays; every
    replay rewrites the outputs and equals the eager solve."""
    import torch

    import paper_1902_04995_amd as rgb
    bt = gen.concat([gen.uneven_batch(2500, m_lo=8, m_hi=3000, seed=34), gen.tiny_random_batch(500, m_max=40, seed=35)])
    dev = rgb.DeviceBatch(bt, "cuda:0")
    ref = _host(dev.solve(variant=variant))
    other = rgb.DeviceBatch(gen.uniform_batch(700, 64, seed=36), "cuda:0")
    other_ref = _host(other.solve(variant=variant))
    out = tuple(torch.empty(bt.num_lps, dtype=dt, device="cuda") for dt in (torch.float32, torch.float32, torch.int32))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream, outside the capture
        rgb.solve_batch_noalloc(dev.offsets, dev.ax, dev.ay, dev.b, dev.cx, dev.cy, out=out, variant=variant,
                                stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rgb.solve_batch_noalloc(dev.offsets, dev.ax, dev.ay, dev.b, dev.cx, dev.cy, out=out, variant=variant,
                                stream=torch.cuda.current_stream())
    for rep in range(3):
        out[0].fill_(7.0)
        out[1].fill_(7.0)
        out[2].fill_(9)
        eager = other.solve(variant=variant)  # eager work of the program between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _same(_host(out), ref, (variant, "replay", rep))
        _same(_host(eager), other_ref, (variant, "eager between replays", rep))
    del g
