"""Benchmark: batched 2D LP solving on one MI355X.

One step = one solve of the whole synthetic workload (every LP of the batch,
inputs resident in HBM).  Prints ONE JSON line with LPs/s of the batched
solver (``value``), the plain one-LP-per-lane kernel on the same buffers,
constraints/s, the HBM roofline of the dominant kernel (algorithmic bytes =
12 B per half-plane + 28 B per LP, over its HIP-event-timed duration), and
the FP64 oracle timed on the host cores as a baseline.

    python bench.py [--steps K] [--warmup W] [--workload uniform|uneven|crowd|plain]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CPU_SAMPLE_S = 10.0  # seconds of oracle work in the cpu_baseline leg
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, public spec

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by the same counters read for a device copy of
# known size (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0 on gfx950); see profiles/.
# Keyed by (kernel, workload) and valid only for the kernel sources whose
# digest is recorded: after any kernel change the figure is reported as null.
MEASURED_TRAFFIC = {
    "sources": "6d141b153fb7f381",
    ('k_group<16>', 'uniform'): 1221830248,
    ('k_group<8>', 'crowd'): 491983607,
    ('k_binned', 'uneven'): 9081419069,
}


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1902_04995_amd", "csrc")
    for f in ("rgb_kernels.hip", "rgb_device.hpp", "rgb_internal.hpp"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

WORKLOADS = {
    "uniform": "131,072 LPs x 256 half-planes (+4 box rows; 5% infeasible, 2% unbounded), FP32",
    "uneven": "200,000 LPs, half-planes log-uniform in [8, 8192] (+box; 5% infeasible, 2% unbounded), FP32",
    "crowd": "262,144 crowd-avoidance LPs, k~U[8,64] neighbours + 16 speed rows, FP32",
    "plain": "1,024 LPs x 64 half-planes (+4 box rows), FP32",
}


def served_leg(rgb, gen, n_requests, load, pool_size=96, seed=0):
    """Poisson stream of requests (1..4096 LPs, 16..2048 rows each, same mix)
    at `load` x the capacity measured with a burst, through (a) the
    continuous-batching server and (b) a FIFO server that solves one request
    at a time with the plain kernel, on the same arrival trace.  Latency =
    completion - scheduled arrival."""
    import numpy as np

    rng = gen.rng_for(5, seed)
    pool = [gen.served_request(rng) for _ in range(pool_size)]
    lps = np.array([r.num_lps for r in pool])

    def run(srv, order, arrivals):
        tickets = []
        t0 = time.perf_counter()
        for k, t_arr in zip(order, arrivals):
            while time.perf_counter() - t0 < t_arr:
                pass
            t_sub = time.perf_counter() - t0
            tickets.append((srv.submit(pool[k], wait=True), t_sub - t_arr, k))
        lat = []
        for t, lag, k in tickets:
            _, _, _, ms = srv.wait(t)
            lat.append(ms + 1e3 * lag)
        wall = time.perf_counter() - t0
        total = int(sum(lps[k] for _, _, k in tickets))
        lat = np.array(lat)
        return {"requests": len(tickets), "lps": total, "wall_s": wall, "lps_per_s": total / wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat.max())}

    served = rgb.Server(n_streams=4, max_batch_lps=16384, hbm_budget=4 << 30, host_ring_mib=1024)
    fifo = rgb.Server(n_streams=1, one_request_per_batch=True, variant="plain", hbm_budget=4 << 30,
                      host_ring_mib=1024)
    # warm-up (pinned buffers, workspaces) and capacity from a burst of the whole pool
    for srv in (served, fifo):
        for t in [srv.submit(r, wait=True) for r in pool[:8]]:
            srv.wait(t)
    t0 = time.perf_counter()
    for t in [served.submit(r, wait=True) for r in pool]:
        served.wait(t)
    capacity = float(lps.sum()) / (time.perf_counter() - t0)
    order = rng.integers(0, pool_size, n_requests)
    rate = load * capacity / float(lps.mean())  # requests per second
    arrivals = gen.poisson_arrivals(rng, n_requests, rate)
    out = {"capacity_lps_per_s": capacity, "offered_load": load, "offered_lps_per_s": load * capacity,
           "request_mix": "n ~ floor(logU[1, 4096]) LPs, m ~ logU[16, 2048] + box rows, 5% infeasible, 2% unbounded",
           "served": run(served, order, arrivals), "plain_fifo": run(fifo, order, arrivals)}
    out["served"]["stats"] = served.stats()
    served.close()
    fifo.close()
    return out


def host_leg(rgb, bt, tuning, reps=3):
    """The transfer-inclusive rate: the workload solved from host memory to
    host memory (rgb_solve_batch_host: chunks through three streams), with
    pinned and with pageable buffers, and a plain host-to-device copy of the
    inputs for scale.  Context only: `value` never includes transfers."""
    import numpy as np
    import torch
    kw = {}  # AUTO: the context's (autotuned) configuration, as in the timed steps
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    args = [pin(bt.offsets)] + [pin(a) for a in (bt.ax, bt.ay, bt.b, bt.cx, bt.cy)]
    out = (torch.empty(bt.num_lps, dtype=torch.float32).pin_memory(),
           torch.empty(bt.num_lps, dtype=torch.float32).pin_memory(),
           torch.empty(bt.num_lps, dtype=torch.int32).pin_memory())
    res = {}
    for name, a, o in (("pinned", args, out), ("pageable", [bt.offsets, bt.ax, bt.ay, bt.b, bt.cx, bt.cy], None)):
        rgb.solve_batch_host(*a, out=o, **kw)  # warm-up: buffers and streams
        ms = [rgb.solve_batch_host(*a, out=o, **kw)[3] for _ in range(reps)]
        best = float(np.median(ms))
        res[name] = {"ms": best, "lps_per_s": bt.num_lps / (best / 1e3)}
    h2d_bytes = sum(t.numel() * t.element_size() for t in args)
    dev = torch.empty(h2d_bytes // 4, dtype=torch.float32, device="cuda")
    flat = torch.empty(h2d_bytes // 4, dtype=torch.float32).pin_memory()
    dev.copy_(flat, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dev.copy_(flat, non_blocking=True)
    torch.cuda.synchronize()
    h2d_ms = (time.perf_counter() - t0) * 1e3 / reps
    res["h2d_probe"] = {"bytes": h2d_bytes, "ms": h2d_ms, "gbs": h2d_bytes / (h2d_ms / 1e3) / 1e9}
    res["configuration"] = (tuning or {}).get("variant", "auto")
    return res


def crowd_leg(rgb, n=262144, steps=10, seed=0):
    """The crowd time step on the device at the crowd workload's size (agents
    uniform at density 1, k ~ U{8..64} neighbours, 16 speed-disc rows): ms per
    step eager (explicit step numbers) and as a replayed HIP graph (device step
    counter), positions reset before each series."""
    import math

    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    side = math.sqrt(n)
    px = (rng.random(n) * side).astype(np.float32)
    py = (rng.random(n) * side).astype(np.float32)
    k = rng.integers(8, 65, n).astype(np.int32)
    ang = rng.random(n) * 2.0 * math.pi
    g = [torch.from_numpy(a.astype(np.float32)).cuda() for a in (np.cos(ang), np.sin(ang))]
    crowd = rgb.Crowd(k, (0.0, 0.0, side, side), radius=0.3, vmax=1.0, dt=0.1, cell=2.0, n_disc=16, seed=seed)
    dpx, dpy = torch.from_numpy(px).cuda(), torch.from_numpy(py).cuda()
    vx = torch.empty(n, dtype=torch.float32, device="cuda")
    vy = torch.empty_like(vx)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    side_stream = torch.cuda.Stream()
    side_stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side_stream):
        for s in range(2):  # warm-up on the stream the graph is captured on
            crowd.step(dpx, dpy, g[0], g[1], vx, vy, st, s, stream=side_stream)
    torch.cuda.synchronize()

    def series(fn):
        dpx.copy_(torch.from_numpy(px))
        dpy.copy_(torch.from_numpy(py))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(side_stream)
        for s in range(steps):
            fn(s)
        e1.record(side_stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    eager_ms = series(lambda s: crowd.step(dpx, dpy, g[0], g[1], vx, vy, st, s, stream=side_stream))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side_stream):
        crowd.step(dpx, dpy, g[0], g[1], vx, vy, st, -1, stream=side_stream)
    torch.cuda.synchronize()
    with torch.cuda.stream(side_stream):
        graph_ms = series(lambda s: graph.replay())
    status = np.bincount(st.cpu().numpy(), minlength=4).tolist()
    crowd.close()
    return {"agents": n, "rows_per_step": int(crowd.num_rows), "steps": steps, "eager_ms_per_step": eager_ms,
            "graph_ms_per_step": graph_ms, "agent_steps_per_s": n / (min(eager_ms, graph_ms) / 1e3),
            "last_step_status_counts": status}


def kernel_name(variant, tuning, lanes=0):
    """The solve kernel a call runs, with the template arguments that tell
    its instances apart (as in the profiler's kernel names)."""
    v = tuning["variant"] if (variant == "auto" and tuning) else variant
    v = "persistent" if v == "auto" else v
    if v == "pooled":
        return f"k_pool<{lanes or tuning['pool_lanes']}, {tuning['pool_rows']}>"
    if v == "batched":
        return f"k_group<{lanes or tuning['batched_lanes']}>"
    return {"persistent": "k_persist", "binned": "k_binned", "plain": "k_plain"}[v]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (AUTO uses the default plan)")
    ap.add_argument("--tune-budget-ms", type=float, default=3000.0)
    ap.add_argument("--served-requests", type=int, default=1500, help="0 skips the served leg")
    ap.add_argument("--served-load", type=float, default=0.7)
    ap.add_argument("--no-host", action="store_true", help="skip the host-to-host (transfer-inclusive) leg")
    ap.add_argument("--no-crowd", action="store_true", help="skip the crowd time-step leg")
    ap.add_argument("--no-seidel3", action="store_true", help="skip the 3D solver leg")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": f"--gpus {args.gpus}: the benchmark measures one GPU only; "
                                   "LPs are independent, so N GPUs would each solve their own LP range"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1902_04995_amd as rgb
    from paper_1902_04995_amd import gen

    t0 = time.time()
    bt = gen.make_config(args.workload, seed=0)
    gen_s = time.time() - t0
    print(f"[bench] generated {args.workload}: {bt.num_lps} LPs, {bt.num_constraints} rows in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    out = (torch.empty(bt.num_lps, dtype=torch.float32, device="cuda"),
           torch.empty(bt.num_lps, dtype=torch.float32, device="cuda"),
           torch.empty(bt.num_lps, dtype=torch.int32, device="cuda"))
    alg_bytes = bt.algorithmic_bytes()
    tuning = None
    if args.variant == "auto" and not args.no_tune:
        t0 = time.time()
        best = dev.autotune(reps=3, budget_ms=args.tune_budget_ms, out=out, stream=stream)
        tuning = best.to_dict()
        print(f"[bench] autotune {time.time() - t0:.1f}s -> {tuning}", file=sys.stderr, flush=True)
    if tuning is None:
        tuning = rgb.context(0).tuning.to_dict()

    def run(variant, steps, warmup, **kw):
        for _ in range(warmup):
            dev.solve(variant=variant, out=out, stream=stream, **kw)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        for a, b in ev:  # create the events so the library can record them
            a.record(stream)
            b.record(stream)
        torch.cuda.synchronize()
        t_start.record(stream)
        for a, b in ev:
            dev.solve(variant=variant, out=out, stream=stream, events=(a, b), **kw)
        t_end.record(stream)
        torch.cuda.synchronize()
        total_ms = t_start.elapsed_time(t_end)
        per = [a.elapsed_time(b) for a, b in ev]
        return total_ms / steps, float(np.mean(per)), float(np.median(per)), per

    kw = dict(lanes_per_lp=args.lanes)
    ms_step, kern_ms, kern_med, per = run(args.variant, args.steps, args.warmup, **kw)
    print(f"[bench] {args.variant}: {ms_step:.3f} ms/step, kernel mean {kern_ms:.3f} ms median {kern_med:.3f} ms",
          file=sys.stderr, flush=True)
    st = out[2].cpu().numpy()
    status_counts = np.bincount(st, minlength=4).tolist()

    # achievable-bandwidth context: a device copy of as many bytes as the solve reads and writes
    n_copy = alg_bytes // 8
    src = torch.empty(n_copy, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_ms = c0.elapsed_time(c1) / 5
    copy_probe = {"bytes_moved": 8 * n_copy, "ms": copy_ms, "gbs": 8 * n_copy / (copy_ms / 1e3) / 1e9}
    del src, dst

    plain = None
    if not args.no_plain:
        p_steps = max(2, min(args.steps, 5))
        p_ms, p_kern, _, _ = run("plain", p_steps, 1)
        plain = {"lps_per_s": bt.num_lps / (p_ms / 1e3), "ms_per_step": p_ms,
                 "hbm_gbs": alg_bytes / (p_kern / 1e3) / 1e9, "steps": p_steps}
        print(f"[bench] plain: {p_ms:.3f} ms/step", file=sys.stderr, flush=True)

    host = None
    if not args.no_host:
        host = host_leg(rgb, bt, tuning)
        print(f"[bench] host path: {json.dumps(host)}", file=sys.stderr, flush=True)

    crowd = None
    if not args.no_crowd:
        crowd = crowd_leg(rgb)
        print(f"[bench] crowd loop: {json.dumps(crowd)}", file=sys.stderr, flush=True)

    seidel3 = None
    if not args.no_seidel3:
        from paper_1902_04995_amd import gen3, seidel3_run
        seidel3 = seidel3_run.measure(rgb, gen3.make_config3("uniform3", seed=0), steps=10)
        print(f"[bench] 3D: {json.dumps(seidel3)}", file=sys.stderr, flush=True)

    served = None
    if args.served_requests > 0:
        served = served_leg(rgb, gen, args.served_requests, args.served_load)
        print(f"[bench] served: {json.dumps({k: v for k, v in served.items() if k in ('served', 'plain_fifo')})}",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = len(os.sched_getaffinity(0))
        # bounded sample: whole passes over the workload on every host core,
        # repeated until about CPU_SAMPLE_S seconds have gone by
        passes, cpu_s = 0, 0.0
        while passes == 0 or cpu_s < CPU_SAMPLE_S:
            t0 = time.perf_counter()
            ref = oracle.solve(bt, threads=threads)
            cpu_s += time.perf_counter() - t0
            passes += 1
        cpu = {"value": passes * bt.num_lps / cpu_s, "unit": "LPs/s", "cores": int(ref["threads"]), "kind": "oracle",
               "sample": f"{passes} passes over all {bt.num_lps} LPs of the workload, FP64 serial Seidel per LP, "
                         f"LPs split over {ref['threads']} threads ({cpu_s:.1f} s)"}
        agree = int((ref["status"] == st).sum())
        cpu["status_agree"] = f"{agree}/{bt.num_lps}"
        print(f"[bench] oracle: {cpu_s:.2f}s on {ref['threads']} threads; status agree {agree}/{bt.num_lps}",
              file=sys.stderr, flush=True)

    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    kname = kernel_name(args.variant, tuning, args.lanes)
    traffic = None
    if kernel_source_digest() == MEASURED_TRAFFIC["sources"]:
        traffic = MEASURED_TRAFFIC.get((kname, args.workload))
    line = {
        "metric": "LPs/sec + achieved HBM GB/s, batched vs plain kernel; p50/p99 served latency",
        "value": bt.num_lps / (ms_step / 1e3),
        "unit": "LPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator, inputs resident in HBM)",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "num_lps": bt.num_lps,
                   "half_planes": bt.num_constraints, "variant": args.variant,
                   "lanes_per_lp": args.lanes, "tuning": tuning},
        "constraints_per_s": bt.num_constraints / (ms_step / 1e3),
        "hbm_gbs": achieved,
        "plain": plain,
        "batched_over_plain": (bt.num_lps / (ms_step / 1e3)) / plain["lps_per_s"] if plain else None,
        "status_counts": status_counts,
        "copy_probe": copy_probe,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_ms_mean": kern_ms, "kernel_ms_median": kern_med},
        "cpu_baseline": cpu,
        "host_path": host,
        "crowd_loop": crowd,
        "seidel3": seidel3,
        "served": served,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
