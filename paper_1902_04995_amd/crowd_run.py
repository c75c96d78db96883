"""Run the crowd time step on the device for a few steps and print the time
per step: agents uniform at density 1 in a square room, k ~ U{8..64}
neighbours, random preferred directions.

    python -m paper_1902_04995_amd.crowd_run --agents 262144 --steps 6 --lanes 8
"""
import argparse
import json
import math
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--agents", type=int, default=262144)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--cell", type=float, default=2.0)
    ap.add_argument("--lanes", type=int, default=0, help="solve with the batched kernel at this width (0: AUTO)")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_1902_04995_amd as rgb
    n = args.agents
    rng = np.random.default_rng(args.seed)
    side = math.sqrt(n)
    px = (rng.random(n) * side).astype(np.float32)
    py = (rng.random(n) * side).astype(np.float32)
    k = np.minimum(rng.integers(8, 65, n), n - 1).astype(np.int32)
    ang = rng.random(n) * 2.0 * math.pi
    gx, gy = (torch.from_numpy(a.astype(np.float32)).cuda() for a in (np.cos(ang), np.sin(ang)))
    crowd = rgb.Crowd(k, (0.0, 0.0, side, side), cell=args.cell, seed=args.seed)
    dpx, dpy = torch.from_numpy(px).cuda(), torch.from_numpy(py).cuda()
    vx = torch.empty(n, dtype=torch.float32, device="cuda")
    vy = torch.empty_like(vx)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    kw = dict(variant="batched", lanes_per_lp=args.lanes) if args.lanes else {}
    crowd.step(dpx, dpy, gx, gy, vx, vy, st, 0, **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(1, args.steps + 1):
        crowd.step(dpx, dpy, gx, gy, vx, vy, st, s, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({"agents": n, "rows_per_step": crowd.num_rows, "steps": args.steps, "ms_per_step": ms,
                      "status_counts": np.bincount(st.cpu().numpy(), minlength=4).tolist()}))
    crowd.close()


if __name__ == "__main__":
    main()
