"""Batched two-dimensional LP solver for MI355X (gfx950).

Thin Python binding over the C ABI in ``include/rgb.h`` (``librgb.so``,
built in-tree by ``build.py``).  Every step of the solve runs in the HIP
kernels; this module only marshals arguments.  PyTorch provides device
memory and streams.  There is no CPU fallback: if the library is missing,
every call raises.

    import torch, paper_1902_04995_amd as rgb
    x, y, status = rgb.solve_batch(offsets, ax, ay, b, cx, cy)   # CUDA tensors

Statuses: OPTIMAL=0, INFEASIBLE=1, UNBOUNDED=2, INVALID=3.
"""
from __future__ import annotations

import ctypes
import os
import threading
import time

OPTIMAL, INFEASIBLE, UNBOUNDED, INVALID = 0, 1, 2, 3
VARIANTS = {"auto": 0, "plain": 1, "batched": 2, "persistent": 3, "binned": 4, "pooled": 5}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgb.so")
_lib = None
_lock = threading.Lock()
_ctx_cache = {}


class RgbError(RuntimeError):
    pass


class _SolveOpts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("lanes_per_lp", ctypes.c_int32), ("pool_wait", ctypes.c_int32),
                ("pool_rows", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("grid", ctypes.c_int32), ("queue_share", ctypes.c_int32),
                ("n_1dlp_out", ctypes.c_void_p), ("ev_begin", ctypes.c_void_p), ("ev_end", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """rgb_tuning_t: a launch configuration (see include/rgb.h)."""
    _fields_ = [("variant", ctypes.c_int32), ("log2_lanes", ctypes.c_int32 * 16), ("batched_lanes", ctypes.c_int32),
                ("queue_share", ctypes.c_int32), ("chunk", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("pool_lanes", ctypes.c_int32), ("pool_wait", ctypes.c_int32), ("pool_rows", ctypes.c_int32),
                ("ms", ctypes.c_float)]

    def to_dict(self):
        return {"variant": {v: k for k, v in VARIANTS.items()}.get(self.variant, self.variant),
                "log2_lanes": list(self.log2_lanes), "batched_lanes": self.batched_lanes,
                "queue_share": self.queue_share, "chunk": self.chunk, "grid": self.grid,
                "pool_lanes": self.pool_lanes, "pool_wait": self.pool_wait, "pool_rows": self.pool_rows,
                "ms": self.ms}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        v = d["variant"]
        t.variant = VARIANTS[v] if isinstance(v, str) else int(v)
        for i, x in enumerate(d["log2_lanes"]):
            t.log2_lanes[i] = int(x)
        t.batched_lanes = int(d["batched_lanes"])
        t.queue_share = int(d["queue_share"])
        t.chunk = int(d["chunk"])
        t.grid = int(d.get("grid", 0))
        t.pool_lanes = int(d.get("pool_lanes", 4))
        t.pool_wait = int(d.get("pool_wait", 2))
        t.pool_rows = int(d.get("pool_rows", 4))
        t.ms = float(d.get("ms", 0.0))
        return t


class _CtxOpts(ctypes.Structure):
    _fields_ = [("tuning_table", ctypes.c_char_p), ("reserved", ctypes.c_int32 * 4)]


class _CrowdOpts(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("vmax", ctypes.c_float), ("dt", ctypes.c_float), ("cell", ctypes.c_float),
                ("n_disc", ctypes.c_int32), ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("n_streams", ctypes.c_int32), ("max_batch_lps", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("variant", ctypes.c_int32), ("one_request_per_batch", ctypes.c_int32),
                ("host_ring_mib", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected_busy", ctypes.c_uint64),
                ("rejected_too_large", ctypes.c_uint64), ("lps_completed", ctypes.c_uint64),
                ("micro_batches", ctypes.c_uint64), ("arena_bytes_in_use", ctypes.c_uint64),
                ("arena_bytes_peak", ctypes.c_uint64), ("pending", ctypes.c_int32), ("in_flight", ctypes.c_int32)]


def lib():
    """Load librgb.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        import torch  # noqa: F401  (binds the process to torch's HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise RgbError(f"{LIB_PATH} is missing: run paper_1902_04995_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.rgb_version.restype = ctypes.c_char_p
        L.rgb_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(_CtxOpts), ctypes.POINTER(P)]
        L.rgb_ctx_create.restype = I32
        L.rgb_ctx_destroy.argtypes = [P]
        L.rgb_ctx_destroy.restype = I32
        L.rgb_ctx_last_error.argtypes = [P]
        L.rgb_ctx_last_error.restype = ctypes.c_char_p
        L.rgb_solve_batch.argtypes = [P, I64, I64] + [P] * 9 + [ctypes.POINTER(_SolveOpts), P]
        L.rgb_solve_batch.restype = I32
        L.rgb_solve_batch_noalloc.argtypes = [P, I64, I64] + [P] * 9 + [ctypes.POINTER(_SolveOpts), P]
        L.rgb_solve_batch_noalloc.restype = I32
        L.rgb_ctx_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.rgb_ctx_get_tuning.restype = I32
        L.rgb_ctx_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.rgb_ctx_set_tuning.restype = I32
        L.rgb_autotune.argtypes = [P, I64, I64] + [P] * 9 + [I32, ctypes.c_double, ctypes.c_char_p, P,
                                                              ctypes.POINTER(Tuning)]
        L.rgb_autotune.restype = I32
        L.rgb_plan_create.argtypes = [P, I64, I64] + [P] * 9 + [ctypes.POINTER(_SolveOpts), ctypes.POINTER(P)]
        L.rgb_plan_create.restype = I32
        L.rgb_plan_launch.argtypes = [P, P]
        L.rgb_plan_launch.restype = I32
        L.rgb_plan_destroy.argtypes = [P]
        L.rgb_plan_destroy.restype = I32
        L.rgb_server_create.argtypes = [P, ctypes.POINTER(_ServerOpts), ctypes.POINTER(P)]
        L.rgb_server_create.restype = I32
        L.rgb_server_submit.argtypes = [P, I64, I64] + [P] * 6 + [ctypes.POINTER(ctypes.c_uint64)]
        L.rgb_server_submit.restype = I32
        L.rgb_server_poll.argtypes = [P, ctypes.c_uint64, I32, P, P, P, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(I32)]
        L.rgb_server_poll.restype = I32
        L.rgb_server_stats.argtypes = [P, ctypes.POINTER(_ServerStats)]
        L.rgb_server_stats.restype = I32
        L.rgb_server_destroy.argtypes = [P]
        L.rgb_server_destroy.restype = I32
        L.rgb_solve_batch_host.argtypes = [P, I64, I64] + [P] * 9 + [ctypes.POINTER(_SolveOpts), I64,
                                                                       ctypes.POINTER(ctypes.c_double)]
        L.rgb_solve_batch_host.restype = I32
        L.rgb_crowd_create.argtypes = [P, I64, P, P, ctypes.POINTER(_CrowdOpts), ctypes.POINTER(P)]
        L.rgb_crowd_create.restype = I32
        L.rgb_crowd_step.argtypes = [P] + [P] * 7 + [I64, ctypes.POINTER(_SolveOpts), P]
        L.rgb_crowd_step.restype = I32
        L.rgb_crowd_num_rows.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
        L.rgb_crowd_num_rows.restype = I32
        L.rgb_crowd_rows.argtypes = [P, P, P, P, P, P]
        L.rgb_crowd_rows.restype = I32
        L.rgb_crowd_destroy.argtypes = [P]
        L.rgb_crowd_destroy.restype = I32
        L.rgb_reduce_bench_run.argtypes = [I32, I32, I64, P, P, P]
        L.rgb_reduce_bench_run.restype = I32
        L.rgb_solve3_batch.argtypes = [P, I64, I64] + [P] * 8 + [ctypes.c_double] + [P] * 4 + [I32, P, P, P]
        L.rgb_solve3_batch.restype = I32
        L.rgb_solven_batch.argtypes = [P, I32, I64, I64] + [P] * 4 + [ctypes.c_double] + [P] * 2 + [I32, P, P, P]
        L.rgb_solven_batch.restype = I32
        _lib = L
    return _lib


class Context:
    """Owns an rgb_ctx_t on one device.  ``tuning_table``: path of a table
    written by rgb_autotune; its entry for this device becomes the AUTO
    configuration."""

    def __init__(self, device: int = 0, tuning_table: str | None = None):
        L = lib()
        h = ctypes.c_void_p()
        opts = _CtxOpts()
        opts.tuning_table = os.fsencode(tuning_table) if tuning_table else None
        rc = L.rgb_ctx_create(int(device), ctypes.byref(opts), ctypes.byref(h))
        if rc != 0:
            raise RgbError(f"rgb_ctx_create({device}, tuning_table={tuning_table!r}) failed: {rc}")
        self.handle = h
        self.device = int(device)

    def check(self, rc: int, what: str):
        if rc != 0:
            msg = lib().rgb_ctx_last_error(self.handle).decode()
            raise RgbError(f"{what} failed ({rc}): {msg}")

    @property
    def tuning(self) -> "Tuning":
        t = Tuning()
        self.check(lib().rgb_ctx_get_tuning(self.handle, ctypes.byref(t)), "rgb_ctx_get_tuning")
        return t

    @tuning.setter
    def tuning(self, t):
        if isinstance(t, dict):
            t = Tuning.from_dict(t)
        self.check(lib().rgb_ctx_set_tuning(self.handle, ctypes.byref(t)), "rgb_ctx_set_tuning")

    def close(self):
        if self.handle:
            lib().rgb_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def context(device: int = 0) -> Context:
    ctx = _ctx_cache.get(device)
    if ctx is None:
        ctx = _ctx_cache[device] = Context(device)
    return ctx


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_tensor(t, name, dtype, device):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check_out(out, B, device):
    """Caller-supplied (x, y, status) outputs: float32, float32, int32, on the
    batch's device, contiguous, B entries each (the kernels write B of each)."""
    import torch
    if len(out) != 3:
        raise ValueError("out must be (x, y, status)")
    for t, name, dt in zip(out, ("x", "y", "status"), (torch.float32, torch.float32, torch.int32)):
        _check_tensor(t, f"out {name}", dt, device)
        if t.numel() != B:
            raise ValueError(f"out {name} holds {t.numel()} entries, the batch has {B} LPs")


def make_opts(variant="auto", lanes_per_lp=0, pool_wait=0, chunk=0, grid=0, n_1dlp=None, events=None,
              queue_share=0, pool_rows=0) -> _SolveOpts:
    o = _SolveOpts()
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.lanes_per_lp = int(lanes_per_lp)
    o.pool_wait = int(pool_wait)
    o.pool_rows = int(pool_rows)
    o.chunk = int(chunk)
    o.grid = int(grid)
    o.queue_share = int(queue_share)
    o.n_1dlp_out = n_1dlp.data_ptr() if n_1dlp is not None else None
    if events is not None:
        o.ev_begin, o.ev_end = (_event_handle(e) for e in events)
    return o


def _event_handle(ev):
    """Raw hipEvent_t of a torch.cuda.Event (created by recording it once)."""
    if not ev.cuda_event:
        ev.record()
    return ev.cuda_event


def solve_batch(offsets, ax, ay, b, cx, cy, *, variant="auto", lanes_per_lp=0, pool_wait=0, chunk=0, grid=0,
                queue_share=0, pool_rows=0, want_n_1dlp=False, out=None, stream=None, ctx: Context | None = None,
                events=None):
    """Solve a CSR-offset SoA batch held in CUDA tensors (offsets int64[B+1];
    ax, ay, b float32[N]; cx, cy float32[B]).  Enqueues on ``stream`` (default:
    torch's current stream) and returns (x, y, status[, n_1dlp]) tensors that
    are valid once that stream has run the work.  ``events`` = (begin, end)
    torch.cuda.Events recorded around the solve kernel alone."""
    import torch
    dev = offsets.device
    if dev.type != "cuda":
        raise ValueError("solve_batch needs CUDA tensors")
    _check_tensor(offsets, "offsets", torch.int64, dev)
    for name, t in (("ax", ax), ("ay", ay), ("b", b), ("cx", cx), ("cy", cy)):
        _check_tensor(t, name, torch.float32, dev)
    B = offsets.numel() - 1
    N = ax.numel()
    if B < 0 or ay.numel() != N or b.numel() != N or cx.numel() != B or cy.numel() != B:
        raise ValueError("inconsistent batch shapes")
    if out is None:
        x = torch.empty(B, dtype=torch.float32, device=dev)
        y = torch.empty(B, dtype=torch.float32, device=dev)
        st = torch.empty(B, dtype=torch.int32, device=dev)
    else:
        _check_out(out, B, dev)
        x, y, st = out
    n1d = torch.empty(B, dtype=torch.int32, device=dev) if want_n_1dlp else None
    ctx = ctx or context(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    opts = make_opts(variant, lanes_per_lp, pool_wait, chunk, grid, n1d, events, queue_share, pool_rows)
    rc = lib().rgb_solve_batch(ctx.handle, B, N, _ptr(offsets), _ptr(ax), _ptr(ay), _ptr(b), _ptr(cx), _ptr(cy),
                               _ptr(x), _ptr(y), _ptr(st), ctypes.byref(opts), ctypes.c_void_p(stream.cuda_stream))
    ctx.check(rc, "rgb_solve_batch")
    if want_n_1dlp:
        return x, y, st, n1d
    return x, y, st


def solve_batch_noalloc(offsets, ax, ay, b, cx, cy, *, out, variant="auto", lanes_per_lp=0, pool_wait=0, chunk=0,
                        grid=0, queue_share=0, pool_rows=0, stream=None, ctx: Context | None = None, events=None):
    """rgb_solve_batch_noalloc: the solve of ``solve_batch`` into the caller's
    ``out=(x, y, status)`` tensors, with no device allocation by the library
    or by this binding (at most 2^20 LPs; calls that overlap on one device
    race on the library's static workspace)."""
    import torch
    dev = offsets.device
    if dev.type != "cuda":
        raise ValueError("solve_batch_noalloc needs CUDA tensors")
    _check_tensor(offsets, "offsets", torch.int64, dev)
    for name, t in (("ax", ax), ("ay", ay), ("b", b), ("cx", cx), ("cy", cy)):
        _check_tensor(t, name, torch.float32, dev)
    B = offsets.numel() - 1
    N = ax.numel()
    if B < 0 or ay.numel() != N or b.numel() != N or cx.numel() != B or cy.numel() != B:
        raise ValueError("inconsistent batch shapes")
    _check_out(out, B, dev)
    x, y, st = out
    ctx = ctx or context(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    opts = make_opts(variant, lanes_per_lp, pool_wait, chunk, grid, None, events, queue_share, pool_rows)
    rc = lib().rgb_solve_batch_noalloc(ctx.handle, B, N, _ptr(offsets), _ptr(ax), _ptr(ay), _ptr(b), _ptr(cx),
                                       _ptr(cy), _ptr(x), _ptr(y), _ptr(st), ctypes.byref(opts),
                                       ctypes.c_void_p(stream.cuda_stream))
    ctx.check(rc, "rgb_solve_batch_noalloc")
    return x, y, st


def _batch_args(offsets, ax, ay, b, cx, cy, out):
    import torch
    dev = offsets.device
    if dev.type != "cuda":
        raise ValueError("needs CUDA tensors")
    _check_tensor(offsets, "offsets", torch.int64, dev)
    for name, t in (("ax", ax), ("ay", ay), ("b", b), ("cx", cx), ("cy", cy)):
        _check_tensor(t, name, torch.float32, dev)
    B = offsets.numel() - 1
    N = ax.numel()
    if B < 0 or ay.numel() != N or b.numel() != N or cx.numel() != B or cy.numel() != B:
        raise ValueError("inconsistent batch shapes")
    if out is None:
        out = (torch.empty(B, dtype=torch.float32, device=dev), torch.empty(B, dtype=torch.float32, device=dev),
               torch.empty(B, dtype=torch.int32, device=dev))
    else:
        _check_out(out, B, dev)
    x, y, st = out
    return dev, B, N, [_ptr(offsets), _ptr(ax), _ptr(ay), _ptr(b), _ptr(cx), _ptr(cy), _ptr(x), _ptr(y), _ptr(st)], out


def autotune(offsets, ax, ay, b, cx, cy, *, reps=3, budget_ms=2000.0, out=None, stream=None,
             ctx: Context | None = None, table_path: str | None = None) -> Tuning:
    """Measure the kernel families and launch shapes on this batch and make the
    fastest one the context's AUTO configuration (rgb_autotune); with
    ``table_path`` the result is merged into that tuning table."""
    import torch
    dev, B, N, args, out = _batch_args(offsets, ax, ay, b, cx, cy, out)
    ctx = ctx or context(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    best = Tuning()
    rc = lib().rgb_autotune(ctx.handle, B, N, *args, int(reps), float(budget_ms),
                            os.fsencode(table_path) if table_path else None, ctypes.c_void_p(stream.cuda_stream),
                            ctypes.byref(best))
    ctx.check(rc, "rgb_autotune")
    return best


class Plan:
    """A solve captured as a HIP graph (rgb_plan_create) over fixed buffers."""

    def __init__(self, offsets, ax, ay, b, cx, cy, *, variant="auto", lanes_per_lp=0, chunk=0, grid=0,
                 queue_share=0, pool_wait=0, pool_rows=0, out=None, want_n_1dlp=False,
                 ctx: Context | None = None):
        import torch
        dev, B, N, args, out = _batch_args(offsets, ax, ay, b, cx, cy, out)
        self.ctx = ctx or context(dev.index or 0)
        self.out = out
        self.n_1dlp = torch.empty(B, dtype=torch.int32, device=dev) if want_n_1dlp else None
        self._keep = (offsets, ax, ay, b, cx, cy)
        opts = make_opts(variant, lanes_per_lp, pool_wait, chunk, grid, self.n_1dlp, None, queue_share, pool_rows)
        h = ctypes.c_void_p()
        rc = lib().rgb_plan_create(self.ctx.handle, B, N, *args, ctypes.byref(opts), ctypes.byref(h))
        self.ctx.check(rc, "rgb_plan_create")
        self.handle = h

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.out[0].device)
        self.ctx.check(lib().rgb_plan_launch(self.handle, ctypes.c_void_p(stream.cuda_stream)), "rgb_plan_launch")
        return self.out

    def close(self):
        if getattr(self, "handle", None):
            lib().rgb_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


ERR_BUSY, ERR_TOO_LARGE, ERR_NOT_FOUND = -4, -5, -6


class ServerBusy(RgbError):
    pass


class RequestTooLarge(RgbError):
    pass


class Server:
    """Continuous-batching LP server (rgb_server_*): requests come from host
    memory (numpy arrays), results go back to host memory."""

    def __init__(self, ctx: Context | None = None, *, hbm_budget=0, n_streams=0, max_batch_lps=0, max_pending=0,
                 variant="auto", one_request_per_batch=False, host_ring_mib=0):
        self.ctx = ctx or context(0)
        o = _ServerOpts()
        o.hbm_budget = int(hbm_budget)
        o.n_streams = int(n_streams)
        o.max_batch_lps = int(max_batch_lps)
        o.max_pending = int(max_pending)
        o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        o.one_request_per_batch = 1 if one_request_per_batch else 0
        o.host_ring_mib = int(host_ring_mib)
        h = ctypes.c_void_p()
        rc = lib().rgb_server_create(self.ctx.handle, ctypes.byref(o), ctypes.byref(h))
        if rc != 0:
            raise RgbError(f"rgb_server_create failed ({rc})")
        self.handle = h
        self._sizes = {}

    def submit(self, batch, wait=False) -> int:
        """Queue a gen.Batch-like request; returns its ticket.  With wait=True
        a full queue or full host rings are waited out instead of raising
        ServerBusy."""
        import numpy as np
        arrs = [np.ascontiguousarray(batch.offsets, dtype=np.int64)] + \
               [np.ascontiguousarray(getattr(batch, f), dtype=np.float32) for f in ("ax", "ay", "b", "cx", "cy")]
        B = arrs[0].shape[0] - 1
        N = arrs[1].shape[0]
        t = ctypes.c_uint64()
        ptrs = [ctypes.c_void_p(a.ctypes.data) for a in arrs]
        while True:
            rc = lib().rgb_server_submit(self.handle, B, N, *ptrs, ctypes.byref(t))
            if rc != ERR_BUSY or not wait:
                break
            time.sleep(50e-6)
        if rc == ERR_BUSY:
            raise ServerBusy("server queue or host rings full")
        if rc == ERR_TOO_LARGE:
            raise RequestTooLarge(f"request of {B} LPs / {N} rows can never fit")
        if rc != 0:
            raise RgbError(f"rgb_server_submit failed ({rc})")
        self._sizes[t.value] = B
        return t.value

    def poll(self, ticket: int, wait_ms: int = 0):
        """None if not done yet, else (x, y, status, latency_ms) as numpy arrays."""
        import numpy as np
        B = self._sizes.get(ticket)
        if B is None:
            raise RgbError(f"unknown ticket {ticket}")
        x = np.empty(B, np.float32)
        y = np.empty(B, np.float32)
        st = np.empty(B, np.int32)
        lat = ctypes.c_double()
        done = ctypes.c_int32()
        rc = lib().rgb_server_poll(self.handle, ctypes.c_uint64(ticket), int(wait_ms), ctypes.c_void_p(x.ctypes.data),
                                   ctypes.c_void_p(y.ctypes.data), ctypes.c_void_p(st.ctypes.data), ctypes.byref(lat),
                                   ctypes.byref(done))
        if rc != 0:
            raise RgbError(f"rgb_server_poll failed ({rc})")
        if not done.value:
            return None
        del self._sizes[ticket]
        return x, y, st, lat.value

    def wait(self, ticket: int):
        return self.poll(ticket, wait_ms=-1)

    def stats(self) -> dict:
        s = _ServerStats()
        rc = lib().rgb_server_stats(self.handle, ctypes.byref(s))
        if rc != 0:
            raise RgbError(f"rgb_server_stats failed ({rc})")
        return {f: getattr(s, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().rgb_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceBatch:
    """A gen.Batch copied to device memory."""

    def __init__(self, batch, device="cuda"):
        import torch
        t = lambda a: torch.from_numpy(a).to(device)
        self.offsets = t(batch.offsets)
        self.ax, self.ay, self.b = t(batch.ax), t(batch.ay), t(batch.b)
        self.cx, self.cy = t(batch.cx), t(batch.cy)
        self.num_lps = batch.num_lps
        self.num_constraints = batch.num_constraints

    def solve(self, **kw):
        return solve_batch(self.offsets, self.ax, self.ay, self.b, self.cx, self.cy, **kw)

    def autotune(self, **kw):
        return autotune(self.offsets, self.ax, self.ay, self.b, self.cx, self.cy, **kw)

    def plan(self, **kw):
        return Plan(self.offsets, self.ax, self.ay, self.b, self.cx, self.cy, **kw)


REDUCE_METHODS = {"lds_atomic": 0, "global_atomic": 1, "dpp": 2, "serial": 3}


def reduce_bench_run(method, contention, values, out=None, stream=None):
    """Segment minima of a device float tensor with one of the reduction
    methods of rgb_reduce_bench_run (contention = segment length)."""
    import torch
    _check_tensor(values, "values", torch.float32, values.device)
    n = values.numel()
    if out is None:
        out = torch.empty(n // int(contention), dtype=torch.float32, device=values.device)
    if stream is None:
        stream = torch.cuda.current_stream(values.device)
    m = REDUCE_METHODS[method] if isinstance(method, str) else int(method)
    rc = lib().rgb_reduce_bench_run(m, int(contention), n, _ptr(values), _ptr(out), ctypes.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RgbError(f"rgb_reduce_bench_run failed ({rc})")
    return out


def solve_batch_host(offsets, ax, ay, b, cx, cy, *, variant="auto", lanes_per_lp=0, pool_wait=0, pool_rows=0,
                     chunk=0, grid=0, queue_share=0, chunk_rows=0, out=None, ctx: Context | None = None):
    """Solve a batch in host memory (numpy arrays or CPU tensors; pinned ones
    are copied by DMA directly) and return (x, y, status, wall_ms) in host
    memory (rgb_solve_batch_host)."""
    import numpy as np

    def host(a, dt):
        if hasattr(a, "numpy"):
            assert a.device.type == "cpu" and a.is_contiguous()
            return a
        return np.ascontiguousarray(a, dtype=dt)

    arrs = [host(offsets, np.int64)] + [host(a, np.float32) for a in (ax, ay, b, cx, cy)]
    B = (arrs[0].numel() if hasattr(arrs[0], "numel") else arrs[0].shape[0]) - 1
    N = arrs[1].numel() if hasattr(arrs[1], "numel") else arrs[1].shape[0]
    if out is None:
        out = (np.empty(B, np.float32), np.empty(B, np.float32), np.empty(B, np.int32))
    addr = lambda a: ctypes.c_void_p(a.data_ptr() if hasattr(a, "data_ptr") else a.ctypes.data)
    ctx = ctx or context(0)
    opts = make_opts(variant, lanes_per_lp, pool_wait, chunk, grid, None, None, queue_share, pool_rows)
    ms = ctypes.c_double()
    rc = lib().rgb_solve_batch_host(ctx.handle, B, N, *[addr(a) for a in arrs], *[addr(a) for a in out],
                                    ctypes.byref(opts), int(chunk_rows), ctypes.byref(ms))
    ctx.check(rc, "rgb_solve_batch_host")
    return out[0], out[1], out[2], ms.value


class Crowd:
    """Crowd time step on the device (rgb_crowd_*): kNN, the agents' LPs,
    the batched solve and the position update, all on one stream."""

    def __init__(self, k, bounds, *, radius=0.3, vmax=1.0, dt=0.1, cell=2.0, n_disc=16, seed=0,
                 ctx: Context | None = None):
        import numpy as np
        self.ctx = ctx or context(0)
        self.k = np.ascontiguousarray(k, dtype=np.int32)
        self.n = int(self.k.shape[0])
        b = np.ascontiguousarray(bounds, dtype=np.float32)
        o = _CrowdOpts()
        o.radius, o.vmax, o.dt, o.cell, o.n_disc, o.seed = radius, vmax, dt, cell, int(n_disc), int(seed)
        self.opts = o
        h = ctypes.c_void_p()
        rc = lib().rgb_crowd_create(self.ctx.handle, self.n, ctypes.c_void_p(self.k.ctypes.data),
                                    ctypes.c_void_p(b.ctypes.data), ctypes.byref(o), ctypes.byref(h))
        if rc != 0:
            raise RgbError(f"rgb_crowd_create failed ({rc})")
        self.handle = h
        r = ctypes.c_int64()
        lib().rgb_crowd_num_rows(self.handle, ctypes.byref(r))
        self.num_rows = r.value

    def step(self, px, py, gx, gy, vx, vy, status, step, stream=None, **solve_kw):
        """One time step; px, py are updated in place, (vx, vy, status) get
        the chosen velocities and the LP statuses (CUDA tensors)."""
        import torch
        for t, dt in ((px, torch.float32), (py, torch.float32), (gx, torch.float32), (gy, torch.float32),
                      (vx, torch.float32), (vy, torch.float32), (status, torch.int32)):
            _check_tensor(t, "crowd array", dt, px.device)
            if t.numel() != self.n:
                raise ValueError("crowd arrays must hold one entry per agent")
        if stream is None:
            stream = torch.cuda.current_stream(px.device)
        opts = make_opts(**solve_kw)
        rc = lib().rgb_crowd_step(self.handle, *[_ptr(t) for t in (px, py, gx, gy, vx, vy, status)], int(step),
                                  ctypes.byref(opts), ctypes.c_void_p(stream.cuda_stream))
        self.ctx.check(rc, "rgb_crowd_step")

    def rows(self, stream=None):
        """The LPs of the last step as CUDA tensors (offsets, ax, ay, b)."""
        import torch
        dev = torch.device("cuda", self.ctx.device)
        offs = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        ax, ay, b = (torch.empty(self.num_rows, dtype=torch.float32, device=dev) for _ in range(3))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        rc = lib().rgb_crowd_rows(self.handle, _ptr(offs), _ptr(ax), _ptr(ay), _ptr(b),
                                  ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RgbError(f"rgb_crowd_rows failed ({rc})")
        return offs, ax, ay, b

    def close(self):
        if getattr(self, "handle", None):
            lib().rgb_crowd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Three-dimensional LPs (rgb_solve3_batch)
# ---------------------------------------------------------------------------

def solve3_batch(offsets, ax, ay, az, b, cx, cy, cz, box, *, lanes_per_lp=0, out=None, stream=None,
                 ctx: Context | None = None, events=None):
    """Solve a batch of 3D LPs held in CUDA tensors (offsets int64[B+1]; ax,
    ay, az, b float32[N]; cx, cy, cz float32[B]) inside the box |x_k| <= box.
    Enqueues on ``stream`` (default: torch's current stream) and returns
    (x, y, z, status) tensors, valid once that stream has run the work.
    ``events`` = (begin, end) torch.cuda.Events recorded around the kernel."""
    import torch
    dev = offsets.device
    if dev.type != "cuda":
        raise ValueError("solve3_batch needs CUDA tensors")
    _check_tensor(offsets, "offsets", torch.int64, dev)
    for name, t in (("ax", ax), ("ay", ay), ("az", az), ("b", b), ("cx", cx), ("cy", cy), ("cz", cz)):
        _check_tensor(t, name, torch.float32, dev)
    B = offsets.numel() - 1
    N = ax.numel()
    if B < 0 or ay.numel() != N or az.numel() != N or b.numel() != N or cx.numel() != B or cy.numel() != B \
            or cz.numel() != B:
        raise ValueError("inconsistent batch shapes")
    if out is None:
        out = tuple(torch.empty(B, dtype=torch.float32, device=dev) for _ in range(3)) + \
            (torch.empty(B, dtype=torch.int32, device=dev),)
    else:
        if len(out) != 4:
            raise ValueError("out must be (x, y, z, status)")
        _check_out(tuple(out[:2]) + (out[3],), B, dev)
        _check_out((out[2], out[2], out[3]), B, dev)
    x, y, z, st = out
    ctx = ctx or context(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    ev = (None, None) if events is None else tuple(_event_handle(e) for e in events)
    rc = lib().rgb_solve3_batch(ctx.handle, B, N, _ptr(offsets), _ptr(ax), _ptr(ay), _ptr(az), _ptr(b), _ptr(cx),
                                _ptr(cy), _ptr(cz), ctypes.c_double(float(box)), _ptr(x), _ptr(y), _ptr(z), _ptr(st),
                                int(lanes_per_lp), ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(ev[0]),
                                ctypes.c_void_p(ev[1]))
    if rc != 0:
        raise RgbError(f"rgb_solve3_batch failed ({rc})")
    return out


class DeviceBatch3:
    """A gen3.Batch3 copied to device memory."""

    def __init__(self, batch, device="cuda"):
        import torch
        t = lambda a: torch.from_numpy(a).to(device)
        self.offsets = t(batch.offsets)
        self.ax, self.ay, self.az, self.b = t(batch.ax), t(batch.ay), t(batch.az), t(batch.b)
        self.cx, self.cy, self.cz = t(batch.cx), t(batch.cy), t(batch.cz)
        self.box = float(batch.box)
        self.num_lps = batch.num_lps
        self.num_constraints = batch.num_constraints

    def solve(self, **kw):
        return solve3_batch(self.offsets, self.ax, self.ay, self.az, self.b, self.cx, self.cy, self.cz, self.box, **kw)


# ---------------------------------------------------------------------------
# LPs in n = 2..5 dimensions (rgb_solven_batch)

def solven_batch(offsets, a, b, c, box, *, lanes_per_lp=0, out=None, stream=None, ctx: Context | None = None,
                 events=None):
    """Solve a batch of n-dimensional LPs held in CUDA tensors (offsets
    int64[B+1]; a float32[n, N] with row i's normal in column i; b
    float32[N]; c float32[n, B]) inside the box |x_k| <= box.  Enqueues on
    ``stream`` (default: torch's current stream) and returns (x, status):
    x float32[n, B], status int32[B], valid once that stream has run the work.
    ``events`` = (begin, end) torch.cuda.Events recorded around the kernel."""
    import torch
    dev = offsets.device
    if dev.type != "cuda":
        raise ValueError("solven_batch needs CUDA tensors")
    _check_tensor(offsets, "offsets", torch.int64, dev)
    for name, t in (("a", a), ("b", b), ("c", c)):
        _check_tensor(t, name, torch.float32, dev)
    if a.dim() != 2 or c.dim() != 2 or a.shape[0] != c.shape[0]:
        raise ValueError("a and c must be (n, N) and (n, B)")
    n = int(a.shape[0])
    B = offsets.numel() - 1
    N = int(a.shape[1])
    if B < 0 or b.numel() != N or c.shape[1] != B:
        raise ValueError("inconsistent batch shapes")
    if out is None:
        out = (torch.empty((n, B), dtype=torch.float32, device=dev), torch.empty(B, dtype=torch.int32, device=dev))
    else:
        if len(out) != 2:
            raise ValueError("out must be (x, status)")
        _check_tensor(out[0], "out x", torch.float32, dev)
        _check_tensor(out[1], "out status", torch.int32, dev)
        if tuple(out[0].shape) != (n, B) or out[1].numel() != B:
            raise ValueError(f"out must hold x ({n}, {B}) and status ({B},)")
    x, st = out
    ctx = ctx or context(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    ev = (None, None) if events is None else tuple(_event_handle(e) for e in events)
    rc = lib().rgb_solven_batch(ctx.handle, n, B, N, _ptr(offsets), _ptr(a), _ptr(b), _ptr(c),
                                ctypes.c_double(float(box)), _ptr(x), _ptr(st), int(lanes_per_lp),
                                ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(ev[0]), ctypes.c_void_p(ev[1]))
    if rc != 0:
        raise RgbError(f"rgb_solven_batch failed ({rc})")
    return out


class DeviceBatchN:
    """A genn.BatchN copied to device memory."""

    def __init__(self, batch, device="cuda"):
        import numpy as np
        import torch
        t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(device)
        self.offsets = t(batch.offsets)
        self.a, self.b, self.c = t(batch.a), t(batch.b), t(batch.c)
        self.box = float(batch.box)
        self.dim = batch.dim
        self.num_lps = batch.num_lps
        self.num_constraints = batch.num_constraints

    def solve(self, **kw):
        return solven_batch(self.offsets, self.a, self.b, self.c, self.box, **kw)
