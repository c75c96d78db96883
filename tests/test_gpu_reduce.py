"""GPU: the reduction microbenchmark's four segment-minimum methods must all
return the exact minima (numpy's, bit for bit) at every contention, for
lengths that end in a partial block."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", ["lds_atomic", "global_atomic", "dpp", "serial"])
def test_segment_minima_exact(method):
    import torch
    import paper_1902_04995_amd as rgb
    rng = np.random.default_rng(7)
    for c in [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 4096]:
        for segs in (1, 37, (1 << 20) // c):
            v = rng.standard_normal(c * segs).astype(np.float32) * np.float32(1e3)
            v[rng.integers(0, v.size, max(1, v.size // 97))] *= np.float32(1e-40)  # some denormals
            dv = torch.from_numpy(v).cuda()
            got = rgb.reduce_bench_run(method, c, dv)
            torch.cuda.synchronize()
            ref = v.reshape(segs, c).min(axis=1)
            assert np.array_equal(got.cpu().numpy(), ref), (method, c, segs)


def test_bad_arguments():
    import torch
    import paper_1902_04995_amd as rgb
    dv = torch.zeros(100, dtype=torch.float32, device="cuda")
    for c in (3, 1, 8192):
        with pytest.raises(rgb.RgbError):
            rgb.reduce_bench_run("dpp", c, dv)  # not a power of two in [2, 4096]
    with pytest.raises(rgb.RgbError):
        rgb.reduce_bench_run("dpp", 64, dv)  # 100 is not a multiple of 64
    with pytest.raises(rgb.RgbError):
        rgb.reduce_bench_run(9, 4, dv)
