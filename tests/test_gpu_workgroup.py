"""Size classes solved one LP per workgroup (log2_lanes = 8: two waves share
the LP's scan and work units, its first rows kept in LDS) against the plain
kernel, bit for bit with the 1D-LP counts, and against the FP64 oracle, in
both class-aware families, with the wide classes starting at several sizes:
LPs below, at and above the LDS row cache, non-finite, parallel and
out-of-range rows, and one LP of 2^20 rows."""
import os

import numpy as np
import pytest

import lpcheck
from paper_1902_04995_amd import gen

pytestmark = pytest.mark.gpu

CACHE = 1650  # rows the workgroup keeps in LDS


def _cases():
    from test_gpu_parity import EDGE_SETS
    return {
        "golden": lambda: lpcheck.golden_batch(os.path.join(lpcheck.GOLDEN, "hand_lps.txt"))[0],
        "tiny_random": lambda: gen.tiny_random_batch(1500, m_max=70, seed=21),
        "tiny_int_boxed": lambda: gen.tiny_integer_batch(1500, m_max=12, K=6, seed=22, boxed=True),
        "uneven_big": lambda: gen.uneven_batch(1200, 8, 8192, seed=23),
        "around_cache": lambda: gen.concat([gen.uniform_batch(6, m, seed=m) for m in
                                            (CACHE - 5, CACHE - 1, CACHE, CACHE + 1, CACHE + 7, 5000, 8192)]),
        "crowd_small": lambda: gen.make_config("crowd", seed=0, scale=0.01),
        "huge": lambda: gen.concat([gen.uniform_batch(3, 40, seed=6), gen.uniform_batch(1, 1 << 20, seed=7),
                                    gen.uniform_batch(5, 300, seed=8)]),
        **{f"edge_{k}": (lambda f=f, k=k: lpcheck.rows_batch(f(), k)) for k, f in EDGE_SETS.items()},
    }


CASES = _cases()


def _host(out):
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("case", sorted(CASES))
def test_workgroup_classes_match_plain_and_oracle(oracle_lib, case):
    import torch

    import paper_1902_04995_amd as rgb
    bt = CASES[case]()
    ref = oracle_lib.solve(bt)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    x, y, st, n1d = dev.solve(variant="plain", want_n_1dlp=True)
    torch.cuda.synchronize()
    base = _host((st, x, y, n1d))
    ctx = rgb.Context(0)
    try:
        for first in (0, 7, 12):  # classes from here up are solved one LP per workgroup
            t = ctx.tuning
            for c in range(16):
                if c >= first:
                    t.log2_lanes[c] = 8
            ctx.tuning = t
            for variant in ("binned", "persistent"):
                print(f"[gpu] case={case} wide from class {first} variant={variant} lps={bt.num_lps}", flush=True)
                x, y, s, n = dev.solve(variant=variant, ctx=ctx, want_n_1dlp=True)
                torch.cuda.synchronize()
                got = _host((s, x, y, n))
                for a, b_, name in zip(got, base, ("status", "x", "y", "n_1dlp")):
                    same = np.array_equal(a, b_, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b_)
                    assert same, (case, first, variant, name, np.flatnonzero(~((a == b_) | (a != a) & (b_ != b_)))[:8])
                bs, bx = lpcheck.compare(got[0], got[1], got[2], ref["status"], ref["x"], ref["y"])
                assert len(bs) == 0 and len(bx) == 0, (case, first, variant, bs[:5], bx[:5])
                bn, _ = lpcheck.compare_n1d(got[3], ref)
                assert len(bn) == 0, (case, first, variant, bn[:5])
    finally:
        ctx.close()
