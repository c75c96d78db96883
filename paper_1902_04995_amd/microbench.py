"""Reduction microbenchmark: segment minima by LDS atomics, device-memory
atomics, DPP butterflies and one lane per segment, at contentions 2..512
(how many work units meet in one bound), on 2^26 values.  Prints one JSON
object: per method and contention the kernel time, values per ns and whether
the result equals numpy's.

    python -m paper_1902_04995_amd.microbench
"""
import json
import sys

import numpy as np


def main(n_log2=26, reps=10):
    import torch

    import paper_1902_04995_amd as rgb
    n = 1 << n_log2
    rng = np.random.default_rng(11)
    v = rng.standard_normal(n).astype(np.float32)
    dv = torch.from_numpy(v).cuda()
    table = {}
    for method in rgb.REDUCE_METHODS:
        table[method] = {}
        for c in [2, 4, 8, 16, 32, 64, 128, 256, 512]:
            out = torch.empty(n // c, dtype=torch.float32, device="cuda")
            for _ in range(2):
                rgb.reduce_bench_run(method, c, dv, out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                rgb.reduce_bench_run(method, c, dv, out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            exact = bool(np.array_equal(out.cpu().numpy(), v.reshape(-1, c).min(axis=1)))
            table[method][c] = {"ms": round(ms, 4), "values_per_ns": round(n / (ms * 1e6), 2), "exact": exact}
            print(f"[reduce] {method} c={c}: {ms:.3f} ms, {n / (ms * 1e6):.1f} values/ns, exact={exact}",
                  file=sys.stderr, flush=True)
    print(json.dumps({"n": n, "reps": reps, "table": table}))


if __name__ == "__main__":
    main()
