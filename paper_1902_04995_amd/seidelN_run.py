"""Time the n-dimensional solver (rgb_solven_batch) on the 4D and 5D
measurement workloads.

    python -m paper_1902_04995_amd.seidelN_run [--workload uniform4] [--steps K] [--lanes 8,16,32]

Generates the seeded workload (65,536 LPs of 128 hyperplanes in 4D, or of 64
in 5D, inside |x_k| <= 1e4), copies it to HBM, and for each lane width runs
two warm-up launches and K timed ones, with HIP events recorded by the library
around the kernel on the launch stream.  Prints one JSON line; ``measure`` is
what ``bench.py`` calls.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

HBM_PEAK_GBS = 8000.0


def measure(rgb, bt, lanes=(8, 16, 32), steps=10, log=None):
    import torch
    dev = rgb.DeviceBatchN(bt, "cuda:0")
    stream = torch.cuda.current_stream()
    n = bt.dim
    out = (torch.empty((n, bt.num_lps), dtype=torch.float32, device="cuda"),
           torch.empty(bt.num_lps, dtype=torch.int32, device="cuda"))
    per = {}
    for g in lanes:
        for _ in range(2):
            dev.solve(lanes_per_lp=g, out=out, stream=stream)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for a, b in evs:
            dev.solve(lanes_per_lp=g, out=out, stream=stream, events=(a, b))
        e1.record(stream)
        torch.cuda.synchronize()
        per[g] = {"ms_per_step": e0.elapsed_time(e1) / steps,
                  "kernel_ms_mean": float(np.mean([a.elapsed_time(b) for a, b in evs]))}
        if log:
            log(f"[seidelN] {n}D lanes {g}: {per[g]['kernel_ms_mean']:.3f} ms per kernel")
    best = min(per, key=lambda g: per[g]["kernel_ms_mean"])
    dev.solve(lanes_per_lp=best, out=out, stream=stream)
    torch.cuda.synchronize()
    status = np.bincount(out[1].cpu().numpy(), minlength=4).tolist()
    alg = bt.algorithmic_bytes()
    k_ms = per[best]["kernel_ms_mean"]
    achieved = alg / (k_ms / 1e3) / 1e9
    return {"workload": f"{bt.num_lps} LPs x {bt.num_constraints // max(1, bt.num_lps)} hyperplanes in {n}D, "
                        f"box {bt.box:g}",
            "dim": n, "num_lps": bt.num_lps, "rows": bt.num_constraints, "lanes_per_lp": best,
            "lps_per_s": bt.num_lps / (per[best]["ms_per_step"] / 1e3), "ms_per_step": per[best]["ms_per_step"],
            "kernel": f"k_seidelN<{n},{best}>", "kernel_ms_mean": k_ms,
            # like the 3D kernel, bound by FP64 instruction issue and latency
            # (the recursion's small solves and short 1D LPs), not by HBM; its
            # bytes over time are context only
            "roofline": {"bound": "alu", "note": "FP64 issue- and latency-bound; HBM figures are context",
                         "hbm_context": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": alg}},
            "by_lanes": {str(g): v for g, v in per.items()}, "status_counts": status, "steps": steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="uniform4", choices=["uniform4", "uniform5"])
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--lanes", default="8,16,32")
    ap.add_argument("--scale", type=float, default=1.0)
    args = ap.parse_args()
    import paper_1902_04995_amd as rgb
    from paper_1902_04995_amd import genn
    bt = genn.make_config_n(args.workload, seed=0, scale=args.scale)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    res = measure(rgb, bt, tuple(int(g) for g in args.lanes.split(",")), args.steps, log)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
