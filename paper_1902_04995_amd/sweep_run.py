"""Throughput against batch size and LP size (the paper's two axes, Sec. 4-5:
batches of up to ~32K LPs, LPs of up to 8,192 rows; the device is full only
when batch x size is large).

    python -m paper_1902_04995_amd.sweep_run [--steps K]

Two sweeps over the uniform recipe (unit normals at uniform angles with
offsets in [1, 2], the 4 box rows, 5% infeasible, 2% unbounded): the batch size at 256 rows per LP, and
the rows per LP at 16,384 LPs.  Every point is generated, copied to HBM,
autotuned (AUTO then runs the configuration the tuner found), solved K times
with HIP events around the solve kernel, and solved K times with the plain
one-LP-per-lane kernel.  Prints one JSON line per point and a final summary
line.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BATCHES = (128, 512, 2048, 8192, 32768, 131072, 524288)
SIZES = (16, 64, 256, 1024, 4096, 8192)


def _time(dev, steps, stream, **kw):
    import torch
    out = (torch.empty(dev.num_lps, dtype=torch.float32, device="cuda"),
           torch.empty(dev.num_lps, dtype=torch.float32, device="cuda"),
           torch.empty(dev.num_lps, dtype=torch.int32, device="cuda"))
    for _ in range(2):
        dev.solve(out=out, stream=stream, **kw)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:  # create the events so the library can record them
        a.record(stream)
        b.record(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for a, b in ev:
        dev.solve(out=out, stream=stream, events=(a, b), **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, float(np.median([a.elapsed_time(b) for a, b in ev]))


def point(rgb, gen, num_lps, m, steps, seed=0):
    import torch
    t0 = time.time()
    bt = gen.uniform_batch(num_lps, m, seed=seed)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    stream = torch.cuda.current_stream()
    best = dev.autotune(reps=3, budget_ms=1000.0, stream=stream)
    step_ms, kernel_ms = _time(dev, steps, stream)
    plain_steps = max(1, min(steps, 3 if num_lps * m > 2e7 else steps))
    plain_ms, _ = _time(dev, plain_steps, stream, variant="plain")
    alg = bt.algorithmic_bytes()
    res = {"num_lps": num_lps, "rows_per_lp": round(bt.num_constraints / num_lps, 1), "variant": best.to_dict()["variant"], "ms_per_step": step_ms,
           "kernel_ms": kernel_ms, "lps_per_s": num_lps / (step_ms / 1e3),
           "rows_per_s": bt.num_constraints / (step_ms / 1e3),
           "hbm_frac": alg / (kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBS, "plain_ms": plain_ms,
           "over_plain": plain_ms / step_ms, "wall_s": time.time() - t0}
    del dev
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    args = ap.parse_args()
    import paper_1902_04995_amd as rgb
    from paper_1902_04995_amd import gen
    out = {"batch_sweep_rows_per_lp": 260, "size_sweep_lps": 16384, "batch": [], "size": []}
    for B in BATCHES:
        r = point(rgb, gen, B, 256, args.steps)
        out["batch"].append(r)
        print(json.dumps({"sweep": "batch", **r}), flush=True)
    for m in SIZES:
        r = point(rgb, gen, 16384, m, args.steps)
        out["size"].append(r)
        print(json.dumps({"sweep": "size", **r}), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
