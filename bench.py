"""Benchmark: batched 2D LP solving on one MI355X.

One step = one solve of the whole synthetic workload (every LP of the batch,
inputs resident in HBM).  The default workload is the uneven batch: 200,000
LPs with half-plane counts log-uniform in [8, 8192], the largest one-GPU
configuration.  Prints ONE JSON line with LPs/s of the batched solver
(``value``, K back-to-back solves), the plain one-LP-per-lane kernel on the
same buffers, constraints/s, the HBM roofline of the dominant kernel
(algorithmic bytes = 12 B per half-plane + 28 B per LP, over its
HIP-event-timed duration), the same solves with a 1 GiB cache flush before
each (cold: median, p10, p90), the uniform 131,072 x 256 batch as a second
workload, and the FP64 oracle timed on the host cores (one thread and all of
them) as a baseline.

    python bench.py [--steps K] [--warmup W] [--workload uneven|uniform|crowd|plain]
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

# Fabric bytes per launch of the dominant kernel (the L2's misses, which the
# last-level MALL cache or HBM serve), from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by the same counters read for a device copy of
# known size (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0 on gfx950); see profiles/.
# Keyed by (kernel, workload) and valid only for the kernel sources whose
# digest is recorded: after any kernel change the figure is reported as null.
MEASURED_TRAFFIC = {
    "sources": "a5f98dfc0bde5125",
    ('k_group<16>', 'uniform'): 889613359,
    ('k_group<8>', 'crowd'): 413600531,
    ('k_binned', 'uneven'): 6004888242,
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


def served_leg(rgb, gen, n_requests, loads, fifo_requests=1500, threads=4, pool_size=128, seed=0):
    """Poisson streams of requests (floor(logU[1, 4096]) LPs, 16..2048 rows
    each, same mix) at each of `loads` x the capacity measured with a burst,
    submitted by `threads` host threads, through the continuous-batching
    server; and the first `fifo_requests` requests of the last stream through
    a FIFO server that solves one request at a time with the plain kernel.
    Latency = completion - scheduled arrival."""
    import threading

    import numpy as np

    rng = gen.rng_for(5, seed)
    pool = [gen.served_request(rng) for _ in range(pool_size)]
    lps = np.array([r.num_lps for r in pool])

    def run(srv, order, arrivals, nthreads):
        lat = [None] * len(order)
        t0 = time.perf_counter()

        def worker(t):
            mine = []
            for i in range(t, len(order), nthreads):
                wait = arrivals[i] - (time.perf_counter() - t0)
                if wait > 3e-4:
                    time.sleep(wait - 2e-4)
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
                t_sub = time.perf_counter() - t0
                mine.append((i, srv.submit(pool[order[i]], wait=True), t_sub - arrivals[i]))
            for i, tk, lag in mine:
                lat[i] = srv.wait(tk)[3] + 1e3 * lag

        ths = [threading.Thread(target=worker, args=(t,)) for t in range(nthreads)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        wall = time.perf_counter() - t0
        total = int(lps[order].sum())
        lat = np.array(lat)
        return {"requests": len(order), "lps": total, "wall_s": wall, "lps_per_s": total / wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat.max())}

    # The submitting threads are Python: a full garbage collection inside one
    # of them stalls its submits for tens of ms (measured: one 51 ms submit
    # call in the first timed stream, none later), which is the harness, not
    # the server.  Everything allocated so far is frozen out of collection for
    # the timed runs.
    import gc
    gc.collect()
    gc.freeze()
    served = rgb.Server(n_streams=4, max_batch_lps=16384, hbm_budget=4 << 30, host_ring_mib=1024)
    fifo = rgb.Server(n_streams=1, one_request_per_batch=True, variant="plain", hbm_budget=4 << 30,
                      host_ring_mib=1024)
    # warm-up (pinned buffers, workspaces), then the capacity: a burst of the whole pool
    for srv in (served, fifo):
        for t in [srv.submit(r, wait=True) for r in pool[:8]]:
            srv.wait(t)
    burst = run(served, np.arange(pool_size), np.zeros(pool_size), threads)
    capacity = burst["lps_per_s"]
    out = {"capacity_lps_per_s": capacity, "submit_threads": threads,
           "request_mix": "n ~ floor(logU[1, 4096]) LPs, m ~ logU[16, 2048] + box rows, 5% infeasible, 2% unbounded",
           "loads": {}}
    for load in loads:
        order = rng.integers(0, pool_size, n_requests)
        rate = load * capacity / float(lps.mean())  # requests per second
        arrivals = gen.poisson_arrivals(rng, n_requests, rate)
        res = run(served, order, arrivals, threads)
        res["offered_lps_per_s"] = load * capacity
        out["loads"][str(load)] = res
        print(f"[bench] served at {load}x: {json.dumps(res)}", file=sys.stderr, flush=True)
    out["served_stats"] = served.stats()
    n = min(fifo_requests, n_requests)
    out["plain_fifo"] = run(fifo, order[:n], arrivals[:n], threads)
    out["plain_fifo"]["trace"] = f"the first {n} requests of the {loads[-1]}x stream"
    served.close()
    fifo.close()
    gc.unfreeze()
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def measure_workload(rgb, gen, name, args, tune=True):
    """Generate `name`, autotune, then: K back-to-back solves between two
    synchronisations (the timed region; per-solve HIP events recorded by the
    library around the solve kernels), K solves each after a 1 GiB flush
    (cold cache), a device copy of the algorithmic byte count, and the plain
    kernel on the same buffers."""
    import numpy as np
    import torch

    t0 = time.time()
    bt = gen.make_config(name, seed=0)
    print(f"[bench] generated {name}: {bt.num_lps} LPs, {bt.num_constraints} rows in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    out = (torch.empty(bt.num_lps, dtype=torch.float32, device="cuda"),
           torch.empty(bt.num_lps, dtype=torch.float32, device="cuda"),
           torch.empty(bt.num_lps, dtype=torch.int32, device="cuda"))
    alg_bytes = bt.algorithmic_bytes()
    ctx = rgb.context(0)
    tuning = None
    if args.variant == "auto" and tune:
        t0 = time.time()
        best = dev.autotune(reps=3, budget_ms=args.tune_budget_ms, out=out, stream=stream)
        tuning = best.to_dict()
        print(f"[bench] autotune {name} {time.time() - t0:.1f}s -> {tuning}", file=sys.stderr, flush=True)
    if tuning is None:
        tuning = ctx.tuning.to_dict()
    kw = dict(lanes_per_lp=args.lanes)
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB, above the 256 MB MALL + L2

    def events(n):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:  # create the events so the library can record them
            a.record(stream)
            b.record(stream)
        return ev

    def run(variant, steps, warmup, cold=False):
        for _ in range(warmup):
            dev.solve(variant=variant, out=out, stream=stream, **kw)
        ev = events(steps)
        torch.cuda.synchronize()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        for a, b in ev:
            if cold:
                flush.fill_(1.0)
            dev.solve(variant=variant, out=out, stream=stream, events=(a, b), **kw)
        t_end.record(stream)
        torch.cuda.synchronize()
        per = [a.elapsed_time(b) for a, b in ev]
        return t_start.elapsed_time(t_end) / steps, per

    ms_step, per = run(args.variant, args.steps, args.warmup)
    _, per_cold = run(args.variant, args.steps, 0, cold=True)
    del flush
    st = out[2].cpu().numpy()
    kern_ms = float(np.mean(per))
    print(f"[bench] {name}/{args.variant}: {ms_step:.3f} ms/step, solve kernels mean {kern_ms:.3f} ms "
          f"(p10 {pct(per, 10):.3f}, p90 {pct(per, 90):.3f}); cold median {pct(per_cold, 50):.3f} ms",
          file=sys.stderr, flush=True)

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
    del src, dst

    plain = None
    if not args.no_plain:
        p_steps = max(2, min(args.steps, 5))
        p_ms, p_per = run("plain", p_steps, 1)
        plain = {"lps_per_s": bt.num_lps / (p_ms / 1e3), "ms_per_step": p_ms,
                 "hbm_gbs": alg_bytes / (float(np.mean(p_per)) / 1e3) / 1e9, "steps": p_steps}
        print(f"[bench] {name}/plain: {p_ms:.3f} ms/step", file=sys.stderr, flush=True)

    kname = kernel_name(args.variant, tuning, args.lanes)
    traffic = None
    if kernel_source_digest() == MEASURED_TRAFFIC["sources"]:
        traffic = MEASURED_TRAFFIC.get((kname, name))
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    cold_med = pct(per_cold, 50)
    res = {
        "workload": f"{name}: {WORKLOADS[name]}", "num_lps": bt.num_lps, "half_planes": bt.num_constraints,
        "ms_per_step": ms_step, "lps_per_s": bt.num_lps / (ms_step / 1e3),
        "constraints_per_s": bt.num_constraints / (ms_step / 1e3),
        "solve_ms": {"mean": kern_ms, "median": pct(per, 50), "p10": pct(per, 10), "p90": pct(per, 90)},
        "cold_solve_ms": {"mean": float(np.mean(per_cold)), "median": cold_med, "p10": pct(per_cold, 10),
                          "p90": pct(per_cold, 90), "flush": "1 GiB device fill before each solve"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
                     "algorithmic_bytes_per_launch": alg_bytes, "kernel_ms_mean": kern_ms,
                     "kernel_ms_median": pct(per, 50),
                     "cold_frac": alg_bytes / (cold_med / 1e3) / 1e9 / HBM_PEAK_GBS},
        "copy_probe": {"bytes_moved": 8 * n_copy, "ms": copy_ms, "gbs": 8 * n_copy / (copy_ms / 1e3) / 1e9},
        "plain": plain,
        "batched_over_plain": (bt.num_lps / (ms_step / 1e3)) / plain["lps_per_s"] if plain else None,
        "status_counts": np.bincount(st, minlength=4).tolist(),
        "tuning": tuning,
    }
    return bt, st, dev, res


def cpu_leg(bt, st):
    """The oracle as it stands on the host cores: whole passes over the
    workload on every core for about CPU_SAMPLE_S seconds, and one thread on
    a fixed sample of the LPs (every 16th) for about as long at most."""
    import numpy as np

    import oracle
    threads = len(os.sched_getaffinity(0))
    passes, cpu_s = 0, 0.0
    while passes == 0 or cpu_s < CPU_SAMPLE_S:
        t0 = time.perf_counter()
        ref = oracle.solve(bt, threads=threads)
        cpu_s += time.perf_counter() - t0
        passes += 1
    sample = bt.subset(np.arange(0, bt.num_lps, 16))
    one_s, one_n = 0.0, 0
    while one_n == 0 or one_s < CPU_SAMPLE_S / 2:
        t0 = time.perf_counter()
        oracle.solve(sample, threads=1)
        one_s += time.perf_counter() - t0
        one_n += sample.num_lps
        if one_s > CPU_SAMPLE_S:
            break
    agree = int((ref["status"] == st).sum())
    cpu = {"value": passes * bt.num_lps / cpu_s, "unit": "LPs/s", "cores": int(ref["threads"]), "kind": "oracle",
           "sample": f"{passes} passes over all {bt.num_lps} LPs of the workload, FP64 serial Seidel per LP, "
                     f"LPs split over {ref['threads']} threads ({cpu_s:.1f} s)",
           "cpu_model": cpu_model(),
           "one_thread": {"value": one_n / one_s, "unit": "LPs/s", "cores": 1,
                          "sample": f"every 16th LP ({sample.num_lps} LPs, {sample.num_constraints} rows), "
                                    f"{one_n // sample.num_lps} pass(es) in {one_s:.1f} s"},
           "status_agree": f"{agree}/{bt.num_lps}"}
    print(f"[bench] oracle: {cpu['value']:.3g} LPs/s on {ref['threads']} threads, {one_n / one_s:.3g} on one; "
          f"status agree {agree}/{bt.num_lps}", file=sys.stderr, flush=True)
    return cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uneven", choices=sorted(WORKLOADS))
    ap.add_argument("--second-workload", default="uniform",
                    help="a second workload timed the same way and reported beside the first ('' skips it)")
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (AUTO uses the default plan)")
    ap.add_argument("--tune-budget-ms", type=float, default=3000.0)
    ap.add_argument("--served-requests", type=int, default=10000, help="0 skips the served leg")
    ap.add_argument("--served-loads", default="0.5,0.7", help="offered loads, as fractions of the burst capacity")
    ap.add_argument("--served-threads", type=int, default=4, help="host threads submitting requests")
    ap.add_argument("--no-host", action="store_true", help="skip the host-to-host (transfer-inclusive) leg")
    ap.add_argument("--no-crowd", action="store_true", help="skip the crowd time-step leg")
    ap.add_argument("--no-seidel3", action="store_true", help="skip the 3D solver leg")
    ap.add_argument("--no-seidelN", action="store_true", help="skip the 4D and 5D solver legs")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": f"--gpus {args.gpus}: the benchmark measures one GPU only; "
                                   "LPs are independent, so N GPUs would each solve their own LP range"}))
        sys.exit(2)

    import torch  # noqa: F401

    import paper_1902_04995_amd as rgb
    from paper_1902_04995_amd import gen

    second = None
    if args.second_workload and args.second_workload != args.workload:
        _, _, _, second = measure_workload(rgb, gen, args.second_workload, args, tune=not args.no_tune)
    bt, st, dev, main_res = measure_workload(rgb, gen, args.workload, args, tune=not args.no_tune)
    tuning = main_res["tuning"]

    host = None
    if not args.no_host:
        host = host_leg(rgb, bt, tuning)
        print(f"[bench] host path: {json.dumps(host)}", file=sys.stderr, flush=True)
    del dev

    crowd = None
    if not args.no_crowd:
        crowd = crowd_leg(rgb)
        print(f"[bench] crowd loop: {json.dumps(crowd)}", file=sys.stderr, flush=True)

    seidel3 = None
    if not args.no_seidel3:
        from paper_1902_04995_amd import gen3, seidel3_run
        seidel3 = seidel3_run.measure(rgb, gen3.make_config3("uniform3", seed=0), steps=10)
        print(f"[bench] 3D: {json.dumps(seidel3)}", file=sys.stderr, flush=True)

    seidelN = None
    if not args.no_seidelN:
        from paper_1902_04995_amd import genn, seidelN_run
        seidelN = {}
        for wl in ("uniform4", "uniform5"):
            seidelN[wl] = seidelN_run.measure(rgb, genn.make_config_n(wl, seed=0), lanes=(4, 8, 16), steps=10)
            print(f"[bench] {wl}: {json.dumps(seidelN[wl])}", file=sys.stderr, flush=True)

    served = None
    if args.served_requests > 0:
        served = served_leg(rgb, gen, args.served_requests, [float(v) for v in args.served_loads.split(",")],
                            threads=args.served_threads)
        print(f"[bench] served plain FIFO: {json.dumps(served['plain_fifo'])}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu else cpu_leg(bt, st)

    ms_step = main_res["ms_per_step"]
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
        "config": {"workload": main_res["workload"], "num_lps": bt.num_lps, "half_planes": bt.num_constraints,
                   "variant": args.variant, "lanes_per_lp": args.lanes, "tuning": tuning},
        "constraints_per_s": main_res["constraints_per_s"],
        "hbm_gbs": main_res["roofline"]["achieved"],
        "solve_ms": main_res["solve_ms"],
        "cold_solve_ms": main_res["cold_solve_ms"],
        "plain": main_res["plain"],
        "batched_over_plain": main_res["batched_over_plain"],
        "status_counts": main_res["status_counts"],
        "copy_probe": main_res["copy_probe"],
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "second_workload": second,
        "host_path": host,
        "crowd_loop": crowd,
        "seidel3": seidel3,
        "seidelN": seidelN,
        "served": served,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
